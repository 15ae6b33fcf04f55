// Block assembly kernel (gfx950, wave64): one workgroup per block G[t x s],
// regular pairs one entry per lane, singular pairs sorted by class and done
// one pair per lane with wave-uniform Sauter-Schwab tables.
#include <hip/hip_runtime.h>

#include "bem_device.h"

namespace bem {
namespace {

using namespace dev;

constexpr double kPad = 1.0e4;       // coordinate of column padding points (weight 0)
constexpr uint16_t kNoPair = 0xffff; // empty slot of the sorted singular list

// LDS layout of one sub-tile (up to TR rows x TC columns; triangle rule of nq
// points padded to nqp with zero weights):
//   ys[nqp][TC][6] column points in block-local coordinates Y = 2 (y - c):
//                  (-2Y0, -2Y1, -2Y2, |Y|^2, w sqrt(g_j), <Y, n_j>), read as
//                  three 16-byte words (broadcast within a wave)
//   rg[10][TR]     row geometry 2 (v0 - c), 2 e1, 2 e2, sqrt(g_i)
//   rule[3][nqp]   s, t, w of the triangle rule
//   cn[3][TC]      column normals
//   ints           rid[TR], rv[3][TR], cid[TC], cv[3][TC], count, bad,
//                  per-class counts[4] and cursors[4]
//   list[TR*TC]    uint16 codes (row | col << 6 | class << 12) of singular pairs
//   sorted[TR*TC + 192]  the same codes grouped by class, each class padded to
//                  a multiple of 64 with kNoPair
// Row points X = 2 (x - c) are built in registers from rg and the rule, so
// that 4 |x - y|^2 = |X|^2 + |Y|^2 + X . (-2Y) costs one add and three FMAs.
struct Lds {
  double *ys, *rg, *rule, *cn;
  int *rid, *rv, *cid, *cv, *count, *bad, *ccount, *cursor;
  uint16_t *list, *sorted;
};

__device__ __forceinline__ Lds carve(double *base, int nqp, int TR, int TC) {
  Lds l;
  l.ys = base;
  l.rg = l.ys + 6 * nqp * TC;
  l.rule = l.rg + 10 * TR;
  l.cn = l.rule + 3 * nqp;
  int *ib = reinterpret_cast<int *>(l.cn + 3 * TC);
  l.rid = ib;
  l.rv = l.rid + TR;
  l.cid = l.rv + 3 * TR;
  l.cv = l.cid + TC;
  l.count = l.cv + 3 * TC;
  l.bad = l.count + 1;
  l.ccount = l.bad + 1;
  l.cursor = l.ccount + 4;
  l.list = reinterpret_cast<uint16_t *>(l.cursor + 4);
  l.sorted = l.list + TR * TC;
  return l;
}

// Sum over the point pairs of one regular entry (sub-tile row rl, column cl):
// sum_b wy_b sum_a wx_a k'(x_a, y_b), where k' omits the factor 1/(4 pi) and,
// for the double layer, the factor 1/2 of the scaled normal distance.
template <int KERNEL, int LAYER, int XC>
__device__ __forceinline__ Acc<KERNEL> regular_entry(const Lds &l, int TR, int TC, int nqp, int rl,
                                                     int cl, double kq) {
  const double D0 = l.rg[0 * TR + rl], D1 = l.rg[1 * TR + rl], D2 = l.rg[2 * TR + rl];
  const double A0 = l.rg[3 * TR + rl], A1 = l.rg[4 * TR + rl], A2 = l.rg[5 * TR + rl];
  const double B0 = l.rg[6 * TR + rl], B1 = l.rg[7 * TR + rl], B2 = l.rg[8 * TR + rl];
  const double SG = l.rg[9 * TR + rl];
  double n0 = 0, n1 = 0, n2 = 0;
  if constexpr (LAYER == BEM_DLP) {
    n0 = l.cn[cl];
    n1 = l.cn[TC + cl];
    n2 = l.cn[2 * TC + cl];
  }
  const double2 *ycol = reinterpret_cast<const double2 *>(l.ys) + 3 * cl;
  const int ystride = 3 * TC;  // double2 per point index
  Acc<KERNEL> acc;
  for (int ch = 0; ch < nqp; ch += XC) {
    double X0[XC], X1[XC], X2[XC], XX[XC], WX[XC], XN[XC];
#pragma unroll
    for (int a = 0; a < XC; ++a) {
      const double s = l.rule[ch + a], t = l.rule[nqp + ch + a], w = l.rule[2 * nqp + ch + a];
      X0[a] = fma(s, A0, fma(t, B0, D0));
      X1[a] = fma(s, A1, fma(t, B1, D1));
      X2[a] = fma(s, A2, fma(t, B2, D2));
      XX[a] = fma(X0[a], X0[a], fma(X1[a], X1[a], X2[a] * X2[a]));
      WX[a] = w * SG;
      if constexpr (LAYER == BEM_DLP) XN[a] = fma(X0[a], n0, fma(X1[a], n1, X2[a] * n2));
    }
    double2 c0 = ycol[0], c1 = ycol[1], c2 = ycol[2];
    for (int kb = 0; kb < nqp; ++kb) {
      // prefetch the next column point while this one is used
      const double2 *yn = ycol + (kb + 1 < nqp ? kb + 1 : kb) * ystride;
      const double2 p0 = yn[0], p1 = yn[1], p2 = yn[2];
      const double M0 = c0.x, M1 = c0.y, M2 = c1.x, YY = c1.y, WY = c2.x, YN = c2.y;
      double ire = 0.0, iim = 0.0;
#pragma unroll
      for (int a = 0; a < XC; ++a) {
        double s = XX[a] + YY;
        s = fma(X0[a], M0, s);
        s = fma(X1[a], M1, s);
        s = fma(X2[a], M2, s);  // s = 4 r^2
        // h ~ 1/(2r); one Newton step gives z = h (3 - s h^2) ~ 1/r
        const double h = __builtin_amdgcn_rsq(s);
        const double t = s * h;
        const double e = fma(-t, h, 3.0);
        const double z = h * e;
        if constexpr (KERNEL == BEM_LAPLACE) {
          if constexpr (LAYER == BEM_SLP) {
            ire = fma(WX[a], z, ire);
          } else {
            const double dn = XN[a] - YN;  // 2 <x - y, n_j>
            ire = fma(WX[a] * dn, z * z * z, ire);
          }
        } else {
          const double kr = kq * s * z;  // kappa r  (kq = kappa / 4)
          double sn, cs;
          sincos_cw(kr, &sn, &cs);
          if constexpr (LAYER == BEM_SLP) {
            const double wz = WX[a] * z;
            ire = fma(wz, cs, ire);
            iim = fma(wz, sn, iim);
          } else {
            const double u = WX[a] * (XN[a] - YN) * z * z * z;
            ire = fma(u, fma(kr, sn, cs), ire);
            iim = fma(u, fma(-kr, cs, sn), iim);
          }
        }
      }
      acc.re = fma(WY, ire, acc.re);
      if constexpr (KERNEL == BEM_HELMHOLTZ) acc.im = fma(WY, iim, acc.im);
      c0 = p0;
      c1 = p1;
      c2 = p2;
    }
  }
  return acc;
}

template <int KERNEL, int LAYER, int XC>
__global__ __launch_bounds__(kThreads, 2) void k_blocks(const BlockArgs a, const int coupling) {
  extern __shared__ double lds_raw[];
  const int tid = threadIdx.x;
  const int b = blockIdx.x;
  const int64_t rp0 = a.row_ptr[b], rp1 = a.row_ptr[b + 1];
  const int64_t cp0 = a.col_ptr[b], cp1 = a.col_ptr[b + 1];
  const int64_t off = a.out_off[b];
  bool ok = rp0 >= 0 && rp0 <= rp1 && rp1 <= a.row_len && cp0 >= 0 && cp0 <= cp1 &&
            cp1 <= a.col_len && off >= 0 && off <= a.out_len;
  const int64_t nr = rp1 - rp0, nc = cp1 - cp0;
  ok = ok && (nr == 0 || nc <= (a.out_len - off) / nr);
  if (!ok) {
    if (tid == 0) atomicOr(a.flags, FLAG_EINVAL);
    return;
  }
  if (nr == 0 || nc == 0) return;
  const int i0 = a.row_idx[rp0];
  if (i0 < 0 || i0 >= a.nt) {
    if (tid == 0) atomicOr(a.flags, FLAG_EINVAL);
    return;
  }
  // block-local origin: first vertex of the first row triangle
  const double cx = a.geo[G_V0X * a.ldg + i0], cy = a.geo[G_V0Y * a.ldg + i0],
               cz = a.geo[G_V0Z * a.ldg + i0];
  const int nqp = a.nq_pad, nq = a.nq, TR = a.tr, TC = a.tc;
  const Lds l = carve(lds_raw, nqp, TR, TC);
  const double kq = 0.25 * a.kappa;
  const double scale = (LAYER == BEM_DLP ? 0.5 : 1.0) * kInv4Pi;
  const int wave = tid / kWave, lane = tid & (kWave - 1);
  const int64_t L = a.ldg;

  for (int k = tid; k < nqp; k += kThreads) {
    const bool real = k < nq;
    l.rule[k] = real ? a.rule[k] : 0.0;
    l.rule[nqp + k] = real ? a.rule[nq + k] : 0.0;
    l.rule[2 * nqp + k] = real ? a.rule[2 * nq + k] : 0.0;
  }

  for (int64_t r0 = 0; r0 < nr; r0 += TR) {
    for (int64_t c0 = 0; c0 < nc; c0 += TC) {
      const int tr = (int)min((int64_t)TR, nr - r0), tc = (int)min((int64_t)TC, nc - c0);
      __syncthreads();  // the previous sub-tile is done with the LDS
      if (tid < 4) l.ccount[tid] = 0, l.cursor[tid] = 0;
      if (tid == 0) *l.count = 0, *l.bad = 0;
      __syncthreads();
      // phase A: triangle ids (validated), vertex ids, row geometry, normals
      for (int k = tid; k < tr + tc; k += kThreads) {
        const bool isrow = k < tr;
        const int id = isrow ? a.row_idx[rp0 + r0 + k] : a.col_idx[cp0 + c0 + (k - tr)];
        if (id < 0 || id >= a.nt) {
          *l.bad = 1;
          continue;
        }
        if (isrow) {
          l.rid[k] = id;
          for (int m = 0; m < 3; ++m) l.rv[m * TR + k] = a.tri[3 * (int64_t)id + m];
          l.rg[0 * TR + k] = 2.0 * (a.geo[G_V0X * L + id] - cx);
          l.rg[1 * TR + k] = 2.0 * (a.geo[G_V0Y * L + id] - cy);
          l.rg[2 * TR + k] = 2.0 * (a.geo[G_V0Z * L + id] - cz);
          for (int m = 0; m < 6; ++m) l.rg[(3 + m) * TR + k] = 2.0 * a.geo[(G_E1X + m) * L + id];
          l.rg[9 * TR + k] = a.geo[G_SG * L + id];
        } else {
          const int cl = k - tr;
          l.cid[cl] = id;
          for (int m = 0; m < 3; ++m) l.cv[m * TC + cl] = a.tri[3 * (int64_t)id + m];
          l.cn[cl] = a.geo[G_NX * L + id];
          l.cn[TC + cl] = a.geo[G_NY * L + id];
          l.cn[2 * TC + cl] = a.geo[G_NZ * L + id];
        }
      }
      __syncthreads();
      if (*l.bad) {
        if (tid == 0) atomicOr(a.flags, FLAG_EINVAL);
        return;
      }
      // phase B: column quadrature points in block-local coordinates
      for (int k = tid; k < tc * nqp; k += kThreads) {
        const int cl = k % tc, q = k / tc;
        const int id = l.cid[cl];
        double P0, P1, P2, W;
        if (q < nq) {
          const double s = l.rule[q], t = l.rule[nqp + q];
          P0 = 2.0 * fma(s, a.geo[G_E1X * L + id], fma(t, a.geo[G_E2X * L + id], a.geo[G_V0X * L + id] - cx));
          P1 = 2.0 * fma(s, a.geo[G_E1Y * L + id], fma(t, a.geo[G_E2Y * L + id], a.geo[G_V0Y * L + id] - cy));
          P2 = 2.0 * fma(s, a.geo[G_E1Z * L + id], fma(t, a.geo[G_E2Z * L + id], a.geo[G_V0Z * L + id] - cz));
          W = l.rule[2 * nqp + q] * a.geo[G_SG * L + id];
        } else {  // padding point: far away, weight 0
          P0 = P1 = P2 = -kPad;
          W = 0.0;
        }
        double *y = l.ys + 6 * ((int64_t)q * TC + cl);
        y[0] = -2.0 * P0;
        y[1] = -2.0 * P1;
        y[2] = -2.0 * P2;
        y[3] = fma(P0, P0, fma(P1, P1, P2 * P2));
        y[4] = W;
        y[5] = fma(P0, l.cn[cl], fma(P1, l.cn[TC + cl], P2 * l.cn[2 * TC + cl]));
      }
      __syncthreads();
      // phase C: regular entries, one per lane; singular ones are listed
      for (int e = tid; e < tr * tc; e += kThreads) {
        const int rl = e % tr, cl = e / tr;
        const int cls = shared_vertex_count(l.rv[rl], l.rv[TR + rl], l.rv[2 * TR + rl], l.cv[cl],
                                            l.cv[TC + cl], l.cv[2 * TC + cl]);
        if (cls) {
          if (coupling) {
            atomicOr(a.flags, FLAG_EINVAL);
          } else {
            l.list[atomicAdd(l.count, 1)] = (uint16_t)(rl | (cl << 6) | (cls << 12));
            atomicAdd(&l.ccount[cls], 1);
          }
          continue;
        }
        Acc<KERNEL> v = regular_entry<KERNEL, LAYER, XC>(l, TR, TC, nqp, rl, cl, kq);
        v.re *= scale;
        if constexpr (KERNEL == BEM_HELMHOLTZ) v.im *= scale;
        store<KERNEL>(a.out, off + (r0 + rl) + nr * (c0 + cl), v, a.flags);
      }
      __syncthreads();
      const int ns = *l.count;
      if (ns == 0) continue;
      // phase D: group the singular pairs by class (identical, edge, vertex),
      // each group padded to a multiple of 64 so that every wave-sized chunk
      // holds one class
      const int n3 = (l.ccount[3] + 63) & ~63, n2 = (l.ccount[2] + 63) & ~63,
                n1 = (l.ccount[1] + 63) & ~63;
      const int seg[4] = {0, n3 + n2, n3, 0};  // start of the group of class c
      const int total = n3 + n2 + n1;
      for (int k = tid; k < total; k += kThreads) l.sorted[k] = kNoPair;
      __syncthreads();
      for (int k = tid; k < ns; k += kThreads) {
        const uint16_t code = l.list[k];
        const int cls = code >> 12;
        l.sorted[seg[cls] + atomicAdd(&l.cursor[cls], 1)] = code;
      }
      __syncthreads();
      // phase E: one singular pair per lane, one class per wave-sized chunk
      for (int chunk = wave; chunk * kWave < total; chunk += kThreads / kWave) {
        const int cls = chunk * kWave < n3 ? CLS_IDENTICAL
                        : chunk * kWave < n3 + n2 ? CLS_EDGE : CLS_VERTEX;
        const uint16_t code = l.sorted[chunk * kWave + lane];
        const bool active = code != kNoPair;
        const int rl = code & 63, cl = (code >> 6) & 63;
        PairGeo g;
        bool have = false;
        if (active) have = pair_geometry(a.v, a.tri, a.nv, a.geo, a.ldg, l.rid[rl], l.cid[cl], cls,
                                         a.flags, &g);
        if (!have) {  // idle lane: harmless finite geometry, result discarded
          for (int c = 0; c < 3; ++c)
            g.E1i[c] = c == 0, g.E2i[c] = c == 1, g.E1j[c] = -(c == 2), g.E2j[c] = 0, g.n[c] = 0;
          g.scale = 0.0;
        }
        const Acc<KERNEL> v = ss_pair_lane<KERNEL, LAYER>(g, a.ss, cls, a.kappa);
        if (have) store<KERNEL>(a.out, off + (r0 + rl) + nr * (c0 + cl), v, a.flags);
      }
    }
  }
}

template <int KERNEL, int LAYER>
hipError_t launch_kl(bool coupling, const BlockArgs &a, size_t lds, hipStream_t s) {
  const dim3 grid(a.nblocks), block(kThreads);
  const int cp = coupling ? 1 : 0;
  switch (rule_chunk(a.nq, KERNEL)) {
    case 4: hipLaunchKernelGGL((k_blocks<KERNEL, LAYER, 4>), grid, block, lds, s, a, cp); break;
    case 5: hipLaunchKernelGGL((k_blocks<KERNEL, LAYER, 5>), grid, block, lds, s, a, cp); break;
    case 7: hipLaunchKernelGGL((k_blocks<KERNEL, LAYER, 7>), grid, block, lds, s, a, cp); break;
    case 8: hipLaunchKernelGGL((k_blocks<KERNEL, LAYER, 8>), grid, block, lds, s, a, cp); break;
    default: hipLaunchKernelGGL((k_blocks<KERNEL, LAYER, 9>), grid, block, lds, s, a, cp); break;
  }
  return hipGetLastError();
}

}  // namespace

// x-points per register chunk: the largest supported divisor of nq that keeps
// the kernel within 256 registers (two waves per SIMD), else 4 with padding.
int rule_chunk(int nq, int kernel) {
  static const int lap[] = {8, 9, 7, 5, 4};
  static const int hel[] = {4, 5, 7, 9, 8};  // sine/cosine chains need more registers
  for (int xc : (kernel == BEM_LAPLACE ? lap : hel))
    if (nq % xc == 0) return xc;
  return 4;
}

size_t block_lds_bytes(int nq_pad, int tr, int tc) {
  const size_t dbl = (size_t)6 * nq_pad * tc + 10 * (size_t)tr + 3 * (size_t)nq_pad + 3 * (size_t)tc;
  const size_t ints = (size_t)4 * tr + 4 * (size_t)tc + 10;
  return dbl * 8 + ints * 4 + (size_t)2 * (2 * (size_t)tr * tc + 192);
}

bool block_tile_shape(int nq_pad, size_t lds_budget, int *tr, int *tc, size_t *lds_bytes) {
  static const int shapes[][2] = {{64, 64}, {64, 32}, {64, 16}, {64, 8}, {32, 8}, {16, 8}, {8, 8}};
  for (auto &sh : shapes) {
    const size_t bytes = block_lds_bytes(nq_pad, sh[0], sh[1]);
    if (bytes <= lds_budget) {
      *tr = sh[0];
      *tc = sh[1];
      *lds_bytes = bytes;
      return true;
    }
  }
  return false;
}

hipError_t launch_blocks(int kernel, int layer, bool coupling, const BlockArgs &a,
                         size_t lds, hipStream_t s) {
  if (a.nblocks == 0) return hipSuccess;
  if (kernel == BEM_LAPLACE)
    return layer == BEM_SLP ? launch_kl<BEM_LAPLACE, BEM_SLP>(coupling, a, lds, s)
                            : launch_kl<BEM_LAPLACE, BEM_DLP>(coupling, a, lds, s);
  return layer == BEM_SLP ? launch_kl<BEM_HELMHOLTZ, BEM_SLP>(coupling, a, lds, s)
                          : launch_kl<BEM_HELMHOLTZ, BEM_DLP>(coupling, a, lds, s);
}

}  // namespace bem
