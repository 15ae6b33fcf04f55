// HIP kernels for gfx950 (CDNA4, wave64): per-triangle geometry, block
// assembly (regular rule + Sauter-Schwab pass) and per-entry evaluation.
#include <hip/hip_runtime.h>

#include "bem_internal.h"

namespace bem {
namespace {

constexpr double kInv4Pi = 0.0795774715459476678844418816863;  // 1 / (4 pi)
constexpr int kThreads = 256;
constexpr int kWave = 64;
constexpr double kPad = 1.0e4;  // coordinate of padding points (weight 0)

// ---------------------------------------------------------------- math
// 1/sqrt(a) for a > 0: hardware estimate (relative error below 6e-8) and one
// Newton step y (3 - a y^2) / 2, which leaves a relative error near 1e-15.
__device__ __forceinline__ double rsqrt_newton(double a) {
  const double y = __builtin_amdgcn_rsq(a);
  const double t = a * y;
  const double e = fma(-t, y, 1.0);
  return fma(0.5 * y, e, y);
}

// sin and cos of x: Cody-Waite reduction x = k pi/2 + r, |r| <= pi/4, with
// pi/2 split into three parts (the first two with 33 significant bits so that
// k * part is exact for |k| < 2^20), then the Taylor polynomials of sin and
// cos on [-pi/4, pi/4] truncated after x^17 / x^18 (remainders below 1e-19),
// and the quadrant of k.
constexpr double kTwoOverPi = 0.63661977236758134308;
constexpr double kPio2a = 1.5707963267341256;        // 0x1.921fb544p+0
constexpr double kPio2b = 6.077100506303966e-11;     // 0x1.0b4611a6p-34
constexpr double kPio2c = 2.0222662487959506e-21;    // 0x1.3198a2e037073p-69

__device__ __forceinline__ void sincos_cw(double x, double *s, double *c) {
  const double k = __builtin_rint(x * kTwoOverPi);
  double r = fma(-k, kPio2a, x);
  r = fma(-k, kPio2b, r);
  r = fma(-k, kPio2c, r);
  const double r2 = r * r;
  double ps = 1.0 / 355687428096000.0;      //  1/17!
  ps = fma(ps, r2, -1.0 / 1307674368000.0); // -1/15!
  ps = fma(ps, r2, 1.0 / 6227020800.0);     //  1/13!
  ps = fma(ps, r2, -1.0 / 39916800.0);      // -1/11!
  ps = fma(ps, r2, 1.0 / 362880.0);         //  1/9!
  ps = fma(ps, r2, -1.0 / 5040.0);          // -1/7!
  ps = fma(ps, r2, 1.0 / 120.0);            //  1/5!
  ps = fma(ps, r2, -1.0 / 6.0);             // -1/3!
  const double sr = fma(r * r2, ps, r);
  double pc = -1.0 / 6402373705728000.0;    // -1/18!
  pc = fma(pc, r2, 1.0 / 20922789888000.0); //  1/16!
  pc = fma(pc, r2, -1.0 / 87178291200.0);   // -1/14!
  pc = fma(pc, r2, 1.0 / 479001600.0);      //  1/12!
  pc = fma(pc, r2, -1.0 / 3628800.0);       // -1/10!
  pc = fma(pc, r2, 1.0 / 40320.0);          //  1/8!
  pc = fma(pc, r2, -1.0 / 720.0);           // -1/6!
  pc = fma(pc, r2, 1.0 / 24.0);             //  1/4!
  pc = fma(pc, r2, -0.5);                   // -1/2!
  const double cr = fma(r2, pc, 1.0);
  const int q = static_cast<int>(k) & 3;
  const double a = (q & 1) ? cr : sr;
  const double b = (q & 1) ? sr : cr;
  *s = (q & 2) ? -a : a;
  *c = ((q + 1) & 2) ? -b : b;
}

template <int KERNEL>
struct Acc;
template <>
struct Acc<BEM_LAPLACE> {
  double re = 0.0;
};
template <>
struct Acc<BEM_HELMHOLTZ> {
  double re = 0.0, im = 0.0;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

template <int KERNEL>
__device__ __forceinline__ void store(void *out, int64_t k, const Acc<KERNEL> &v, unsigned *flags) {
  if constexpr (KERNEL == BEM_LAPLACE) {
    if (!isfinite(v.re)) atomicOr(flags, FLAG_NONFINITE);
    static_cast<double *>(out)[k] = v.re;
  } else {
    if (!isfinite(v.re) || !isfinite(v.im)) atomicOr(flags, FLAG_NONFINITE);
    static_cast<double2 *>(out)[k] = make_double2(v.re, v.im);
  }
}

__device__ __forceinline__ int shared_vertex_count(int a0, int a1, int a2, int b0, int b1, int b2) {
  return (a0 == b0) + (a0 == b1) + (a0 == b2) + (a1 == b0) + (a1 == b1) + (a1 == b2) +
         (a2 == b0) + (a2 == b1) + (a2 == b2);
}

// ---------------------------------------------------------- Sauter-Schwab
// Relabelling of a singular pair (common vertices first):
//   identical: mesh order; edge: common vertices (lo, hi) by global id, then
//   the third; vertex: the common vertex, then the rest in cyclic order.
__device__ __forceinline__ void relabel(const int ti[3], const int tj[3], int cls, int li[3],
                                        int lj[3]) {
  if (cls == CLS_IDENTICAL) {
    for (int k = 0; k < 3; ++k) li[k] = ti[k], lj[k] = tj[k];
    return;
  }
  if (cls == CLS_EDGE) {
    int c0 = -1, c1 = -1;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        if (ti[a] == tj[b]) {
          if (c0 < 0) c0 = ti[a]; else c1 = ti[a];
        }
    const int lo = min(c0, c1), hi = max(c0, c1);
    int ci = ti[0], cj = tj[0];
    for (int k = 0; k < 3; ++k) {
      if (ti[k] != lo && ti[k] != hi) ci = ti[k];
      if (tj[k] != lo && tj[k] != hi) cj = tj[k];
    }
    li[0] = lo, li[1] = hi, li[2] = ci;
    lj[0] = lo, lj[1] = hi, lj[2] = cj;
    return;
  }
  int ka = 0, kb = 0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      if (ti[a] == tj[b]) ka = a, kb = b;
  for (int k = 0; k < 3; ++k) li[k] = ti[(ka + k) % 3], lj[k] = tj[(kb + k) % 3];
}

// One singular pair, computed by a whole wave: lanes stride over the rule's
// points, then a butterfly sum.  Every lane returns the entry.
template <int KERNEL, int LAYER>
__device__ Acc<KERNEL> ss_pair_wave(const double *v, const int32_t *tri, int nv, const double *geo,
                                    int64_t ldg, const double *const ss[4], const int32_t np[4],
                                    double kappa, int i, int j, int cls, unsigned *flags) {
  const int lane = threadIdx.x & (kWave - 1);
  int ti[3], tj[3], li[3], lj[3];
  bool ok = true;
  for (int k = 0; k < 3; ++k) {
    ti[k] = tri[3 * (int64_t)i + k];
    tj[k] = tri[3 * (int64_t)j + k];
    ok = ok && ti[k] >= 0 && ti[k] < nv && tj[k] >= 0 && tj[k] < nv;
  }
  Acc<KERNEL> res;
  if (!ok) {
    if (lane == 0) atomicOr(flags, FLAG_EINVAL);
    return res;
  }
  relabel(ti, tj, cls, li, lj);
  double pi[3][3], pj[3][3];
  for (int k = 0; k < 3; ++k)
    for (int c = 0; c < 3; ++c) {
      pi[k][c] = v[3 * (int64_t)li[k] + c];
      pj[k][c] = v[3 * (int64_t)lj[k] + c];
    }
  double D[3], E1i[3], E2i[3], E1j[3], E2j[3];
  for (int c = 0; c < 3; ++c) {
    D[c] = pi[0][c] - pj[0][c];  // zero: both maps start at a common vertex
    E1i[c] = pi[1][c] - pi[0][c];
    E2i[c] = pi[2][c] - pi[1][c];
    E1j[c] = pj[1][c] - pj[0][c];
    E2j[c] = pj[2][c] - pj[1][c];
  }
  const double nx = geo[G_NX * ldg + j], ny = geo[G_NY * ldg + j], nz = geo[G_NZ * ldg + j];
  const double *T = ss[cls];
  const int n = np[cls];
  double are = 0.0, aim = 0.0;
  for (int p = lane; p < n; p += kWave) {
    const double xs = T[p], xt = T[n + p], ys = T[2 * n + p], yt = T[3 * n + p], w = T[4 * n + p];
    double d[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      d[c] = fma(-yt, E2j[c], fma(-ys, E1j[c], fma(xt, E2i[c], fma(xs, E1i[c], D[c]))));
    const double r2 = fma(d[0], d[0], fma(d[1], d[1], d[2] * d[2]));
    const double z = rsqrt_newton(r2);
    double k = z;
    if constexpr (LAYER == BEM_DLP) k = fma(d[0], nx, fma(d[1], ny, d[2] * nz)) * z * z * z;
    if constexpr (KERNEL == BEM_LAPLACE) {
      are = fma(w, k, are);
    } else {
      double sn, cs;
      const double kr = kappa * r2 * z;
      sincos_cw(kr, &sn, &cs);
      if constexpr (LAYER == BEM_SLP) {
        are = fma(w * k, cs, are);
        aim = fma(w * k, sn, aim);
      } else {  // e^{ikr} (1 - i kr)
        are = fma(w * k, fma(kr, sn, cs), are);
        aim = fma(w * k, fma(-kr, cs, sn), aim);
      }
    }
  }
  const double scale = geo[G_SG * ldg + i] * geo[G_SG * ldg + j] * kInv4Pi;
  res.re = wave_sum(are) * scale;
  if constexpr (KERNEL == BEM_HELMHOLTZ) res.im = wave_sum(aim) * scale;
  return res;
}

// ---------------------------------------------------------------- geometry
__global__ void k_geometry(const double *v, int32_t nv, const int32_t *tri, int32_t nt,
                           double *geo, int64_t ldg, unsigned *flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nt) return;
  const int a = tri[3 * (int64_t)i], b = tri[3 * (int64_t)i + 1], c = tri[3 * (int64_t)i + 2];
  double out[GEO_NF];
  for (int f = 0; f < GEO_NF; ++f) out[f] = 0.0;
  if (a < 0 || a >= nv || b < 0 || b >= nv || c < 0 || c >= nv) {
    atomicOr(flags, FLAG_EINVAL);
  } else {
    double p0[3], p1[3], p2[3];
    for (int k = 0; k < 3; ++k) {
      p0[k] = v[3 * (int64_t)a + k];
      p1[k] = v[3 * (int64_t)b + k];
      p2[k] = v[3 * (int64_t)c + k];
    }
    double e1[3], e2[3];
    for (int k = 0; k < 3; ++k) e1[k] = p1[k] - p0[k], e2[k] = p2[k] - p1[k];
    const double n0 = e1[1] * e2[2] - e1[2] * e2[1];
    const double n1 = e1[2] * e2[0] - e1[0] * e2[2];
    const double n2 = e1[0] * e2[1] - e1[1] * e2[0];
    const double sg = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
    if (!(sg > 0.0) || !isfinite(sg)) atomicOr(flags, FLAG_EINVAL);
    for (int k = 0; k < 3; ++k) {
      out[G_V0X + k] = p0[k];
      out[G_E1X + k] = e1[k];
      out[G_E2X + k] = e2[k];
      out[G_LOX + k] = fmin(p0[k], fmin(p1[k], p2[k]));
      out[G_HIX + k] = fmax(p0[k], fmax(p1[k], p2[k]));
    }
    out[G_SG] = sg;
    out[G_NX] = n0 / sg;
    out[G_NY] = n1 / sg;
    out[G_NZ] = n2 / sg;
  }
  for (int f = 0; f < GEO_NF; ++f) geo[f * ldg + i] = out[f];
}

// ---------------------------------------------------------------- blocks
// LDS layout of one sub-tile (tr rows x tc columns, rules padded to nqp):
//   xs[5][nqp][tr]: row points in block-local coordinates X = 2 (x - c):
//                   X0, X1, X2, |X|^2, weight * sqrt(g)
//   ys[6][nqp][tc]: column points Y = 2 (y - c): -2Y0, -2Y1, -2Y2, |Y|^2,
//                   weight * sqrt(g), <Y, n_j>
//   cn[3][tc]:      column normals
//   ints: rid[tr], rv[3][tr], cid[tc], cv[3][tc], list[tr*tc], count, bad
// With these, 4 |x - y|^2 = |X|^2 + |Y|^2 + X . (-2Y) takes one add and
// three FMAs per point pair.
struct Lds {
  double *xs, *ys, *cn;
  int *rid, *rv, *cid, *cv, *list, *count, *bad;
};

__device__ __forceinline__ Lds carve(double *base, int nqp, int tr, int tc) {
  Lds l;
  l.xs = base;
  l.ys = l.xs + 5 * nqp * tr;
  l.cn = l.ys + 6 * nqp * tc;
  int *ib = reinterpret_cast<int *>(l.cn + 3 * tc);
  l.rid = ib;
  l.rv = l.rid + tr;
  l.cid = l.rv + 3 * tr;
  l.cv = l.cid + tc;
  l.list = l.cv + 3 * tc;
  l.count = l.list + tr * tc;
  l.bad = l.count + 1;
  return l;
}

// Sum over all point pairs of one regular entry (row rl, column cl of the
// sub-tile).  Returns sum_b wy_b sum_a wx_a k'(a, b) where k' is the kernel
// without the constant 1/(4 pi) (and for the DLP without the factor 1/2 of
// the scaled normal distance).
template <int KERNEL, int LAYER, int XC>
__device__ __forceinline__ Acc<KERNEL> regular_sum(const Lds &l, int nqp, int tr, int tc, int rl,
                                                   int cl, double kq) {
  Acc<KERNEL> acc;
  double n0 = 0, n1 = 0, n2 = 0;
  if constexpr (LAYER == BEM_DLP) {
    n0 = l.cn[cl];
    n1 = l.cn[tc + cl];
    n2 = l.cn[2 * tc + cl];
  }
  for (int ch = 0; ch < nqp; ch += XC) {
    double X0[XC], X1[XC], X2[XC], XX[XC], WX[XC], XN[XC];
#pragma unroll
    for (int a = 0; a < XC; ++a) {
      const int k = ch + a;
      X0[a] = l.xs[(0 * nqp + k) * tr + rl];
      X1[a] = l.xs[(1 * nqp + k) * tr + rl];
      X2[a] = l.xs[(2 * nqp + k) * tr + rl];
      XX[a] = l.xs[(3 * nqp + k) * tr + rl];
      WX[a] = l.xs[(4 * nqp + k) * tr + rl];
      if constexpr (LAYER == BEM_DLP) XN[a] = fma(X0[a], n0, fma(X1[a], n1, X2[a] * n2));
    }
    for (int kb = 0; kb < nqp; ++kb) {
      const double M0 = l.ys[(0 * nqp + kb) * tc + cl];
      const double M1 = l.ys[(1 * nqp + kb) * tc + cl];
      const double M2 = l.ys[(2 * nqp + kb) * tc + cl];
      const double YY = l.ys[(3 * nqp + kb) * tc + cl];
      const double WY = l.ys[(4 * nqp + kb) * tc + cl];
      double YN = 0.0;
      if constexpr (LAYER == BEM_DLP) YN = l.ys[(5 * nqp + kb) * tc + cl];
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
    }
  }
  return acc;
}

template <int KERNEL, int LAYER, int XC>
__global__ __launch_bounds__(kThreads) void k_blocks(const BlockArgs a, const int coupling) {
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
  const double c0x = a.geo[G_V0X * a.ldg + i0], c0y = a.geo[G_V0Y * a.ldg + i0],
               c0z = a.geo[G_V0Z * a.ldg + i0];
  const int nqp = a.nq_pad, nq = a.nq, TR = a.tr, TC = a.tc;
  const Lds l = carve(lds_raw, nqp, TR, TC);
  const double kq = 0.25 * a.kappa;
  const double scale = (LAYER == BEM_DLP ? 0.5 : 1.0) * kInv4Pi;
  const int wave = tid / kWave, lane = tid & (kWave - 1);

  for (int64_t r0 = 0; r0 < nr; r0 += TR) {
    for (int64_t c0 = 0; c0 < nc; c0 += TC) {
      const int tr = (int)min<int64_t>(TR, nr - r0), tc = (int)min<int64_t>(TC, nc - c0);
      __syncthreads();  // previous sub-tile finished with the LDS
      if (tid == 0) *l.count = 0, *l.bad = 0;
      __syncthreads();
      // phase A: triangle ids (validated) and vertex ids
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
        } else {
          const int cl = k - tr;
          l.cid[cl] = id;
          for (int m = 0; m < 3; ++m) l.cv[m * TC + cl] = a.tri[3 * (int64_t)id + m];
          l.cn[cl] = a.geo[G_NX * a.ldg + id];
          l.cn[TC + cl] = a.geo[G_NY * a.ldg + id];
          l.cn[2 * TC + cl] = a.geo[G_NZ * a.ldg + id];
        }
      }
      __syncthreads();
      if (*l.bad) {
        if (tid == 0) atomicOr(a.flags, FLAG_EINVAL);
        return;
      }
      // phase B: quadrature points of rows and columns in local coordinates
      for (int k = tid; k < (tr + tc) * nqp; k += kThreads) {
        const bool isrow = k < tr * nqp;
        const int kk = isrow ? k : k - tr * nqp;
        const int n = isrow ? tr : tc;
        const int sl = kk % n, q = kk / n;
        const int id = isrow ? l.rid[sl] : l.cid[sl];
        double P0, P1, P2, W;
        if (q < nq) {
          const double s = a.rule[q], t = a.rule[nq + q], w = a.rule[2 * nq + q];
          const double dx = a.geo[G_V0X * a.ldg + id] - c0x;
          const double dy = a.geo[G_V0Y * a.ldg + id] - c0y;
          const double dz = a.geo[G_V0Z * a.ldg + id] - c0z;
          P0 = 2.0 * fma(s, a.geo[G_E1X * a.ldg + id], fma(t, a.geo[G_E2X * a.ldg + id], dx));
          P1 = 2.0 * fma(s, a.geo[G_E1Y * a.ldg + id], fma(t, a.geo[G_E2Y * a.ldg + id], dy));
          P2 = 2.0 * fma(s, a.geo[G_E1Z * a.ldg + id], fma(t, a.geo[G_E2Z * a.ldg + id], dz));
          W = w * a.geo[G_SG * a.ldg + id];
        } else {  // padding point: far away, weight 0 (rows +pad, columns -pad)
          P0 = P1 = P2 = isrow ? kPad : -kPad;
          W = 0.0;
        }
        const double PP = fma(P0, P0, fma(P1, P1, P2 * P2));
        if (isrow) {
          l.xs[(0 * nqp + q) * TR + sl] = P0;
          l.xs[(1 * nqp + q) * TR + sl] = P1;
          l.xs[(2 * nqp + q) * TR + sl] = P2;
          l.xs[(3 * nqp + q) * TR + sl] = PP;
          l.xs[(4 * nqp + q) * TR + sl] = W;
        } else {
          l.ys[(0 * nqp + q) * TC + sl] = -2.0 * P0;
          l.ys[(1 * nqp + q) * TC + sl] = -2.0 * P1;
          l.ys[(2 * nqp + q) * TC + sl] = -2.0 * P2;
          l.ys[(3 * nqp + q) * TC + sl] = PP;
          l.ys[(4 * nqp + q) * TC + sl] = W;
          if (LAYER == BEM_DLP)
            l.ys[(5 * nqp + q) * TC + sl] =
                fma(P0, l.cn[sl], fma(P1, l.cn[TC + sl], P2 * l.cn[2 * TC + sl]));
        }
      }
      __syncthreads();
      // phase C: regular entries, one per lane; singular ones are listed
      for (int e = tid; e < tr * tc; e += kThreads) {
        const int rl = e % tr, cl = e / tr;
        const int cnt = shared_vertex_count(l.rv[rl], l.rv[TR + rl], l.rv[2 * TR + rl], l.cv[cl],
                                            l.cv[TC + cl], l.cv[2 * TC + cl]);
        if (cnt) {
          if (coupling) {
            atomicOr(a.flags, FLAG_EINVAL);
          } else {
            const int pos = atomicAdd(l.count, 1);
            l.list[pos] = rl | (cl << 16);
          }
          continue;
        }
        Acc<KERNEL> v = regular_sum<KERNEL, LAYER, XC>(l, nqp, TR, TC, rl, cl, kq);
        v.re *= scale;
        if constexpr (KERNEL == BEM_HELMHOLTZ) v.im *= scale;
        store<KERNEL>(a.out, off + (r0 + rl) + nr * (c0 + cl), v, a.flags);
      }
      __syncthreads();
      // phase D: singular pairs, one wave per pair
      const int ns = *l.count;
      for (int it = wave; it < ns; it += kThreads / kWave) {
        const int code = l.list[it];
        const int rl = code & 0xffff, cl = code >> 16;
        const int i = l.rid[rl], j = l.cid[cl];
        const int cls = shared_vertex_count(l.rv[rl], l.rv[TR + rl], l.rv[2 * TR + rl], l.cv[cl],
                                            l.cv[TC + cl], l.cv[2 * TC + cl]);
        const Acc<KERNEL> v = ss_pair_wave<KERNEL, LAYER>(a.v, a.tri, a.nv, a.geo, a.ldg, a.ss,
                                                          a.ss_np, a.kappa, i, j, cls, a.flags);
        if (lane == 0) store<KERNEL>(a.out, off + (r0 + rl) + nr * (c0 + cl), v, a.flags);
      }
    }
  }
}

// ---------------------------------------------------------------- entries
// Arbitrary (i, j) list: one lane per regular entry with its points computed
// on the fly; singular entries are listed and done by whole waves.
template <int KERNEL, int LAYER>
__global__ __launch_bounds__(kThreads) void k_entries(const EntryArgs a) {
  __shared__ int list[kThreads];
  __shared__ int count;
  const int tid = threadIdx.x;
  if (tid == 0) count = 0;
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * kThreads + tid;
  if (e < a.n) {
    const int i = a.rows[e], j = a.cols[e];
    if (i < 0 || i >= a.nt || j < 0 || j >= a.nt) {
      atomicOr(a.flags, FLAG_EINVAL);
    } else {
      const int cls = shared_vertex_count(a.tri[3 * (int64_t)i], a.tri[3 * (int64_t)i + 1],
                                          a.tri[3 * (int64_t)i + 2], a.tri[3 * (int64_t)j],
                                          a.tri[3 * (int64_t)j + 1], a.tri[3 * (int64_t)j + 2]);
      if (cls) {
        list[atomicAdd(&count, 1)] = tid;
      } else {
        const double *g = a.geo;
        const int64_t L = a.ldg;
        double D[3], E1i[3], E2i[3], E1j[3], E2j[3];
        for (int c = 0; c < 3; ++c) {
          D[c] = g[(G_V0X + c) * L + i] - g[(G_V0X + c) * L + j];
          E1i[c] = g[(G_E1X + c) * L + i];
          E2i[c] = g[(G_E2X + c) * L + i];
          E1j[c] = g[(G_E1X + c) * L + j];
          E2j[c] = g[(G_E2X + c) * L + j];
        }
        const double nx = g[G_NX * L + j], ny = g[G_NY * L + j], nz = g[G_NZ * L + j];
        const int nq = a.nq;
        const double *R = a.rule;
        double are = 0.0, aim = 0.0;
        for (int qa = 0; qa < nq; ++qa) {
          double x[3];
          for (int c = 0; c < 3; ++c) x[c] = fma(R[qa], E1i[c], fma(R[nq + qa], E2i[c], D[c]));
          double ire = 0.0, iim = 0.0;
          for (int qb = 0; qb < nq; ++qb) {
            double d[3];
            for (int c = 0; c < 3; ++c)
              d[c] = fma(-R[qb], E1j[c], fma(-R[nq + qb], E2j[c], x[c]));
            const double r2 = fma(d[0], d[0], fma(d[1], d[1], d[2] * d[2]));
            const double z = rsqrt_newton(r2);
            double k = z;
            if constexpr (LAYER == BEM_DLP) k = fma(d[0], nx, fma(d[1], ny, d[2] * nz)) * z * z * z;
            const double w = R[2 * nq + qb];
            if constexpr (KERNEL == BEM_LAPLACE) {
              ire = fma(w, k, ire);
            } else {
              const double kr = a.kappa * r2 * z;
              double sn, cs;
              sincos_cw(kr, &sn, &cs);
              if constexpr (LAYER == BEM_SLP) {
                ire = fma(w * k, cs, ire);
                iim = fma(w * k, sn, iim);
              } else {
                ire = fma(w * k, fma(kr, sn, cs), ire);
                iim = fma(w * k, fma(-kr, cs, sn), iim);
              }
            }
          }
          are = fma(R[2 * nq + qa], ire, are);
          aim = fma(R[2 * nq + qa], iim, aim);
        }
        const double scale = g[G_SG * L + i] * g[G_SG * L + j] * kInv4Pi;
        Acc<KERNEL> v;
        v.re = are * scale;
        if constexpr (KERNEL == BEM_HELMHOLTZ) v.im = aim * scale;
        store<KERNEL>(a.out, e, v, a.flags);
      }
    }
  }
  __syncthreads();
  const int ns = count, wave = tid / kWave, lane = tid & (kWave - 1);
  for (int it = wave; it < ns; it += kThreads / kWave) {
    const int64_t ee = (int64_t)blockIdx.x * kThreads + list[it];
    const int i = a.rows[ee], j = a.cols[ee];
    const int cls = shared_vertex_count(a.tri[3 * (int64_t)i], a.tri[3 * (int64_t)i + 1],
                                        a.tri[3 * (int64_t)i + 2], a.tri[3 * (int64_t)j],
                                        a.tri[3 * (int64_t)j + 1], a.tri[3 * (int64_t)j + 2]);
    const Acc<KERNEL> v = ss_pair_wave<KERNEL, LAYER>(a.v, a.tri, a.nv, a.geo, a.ldg, a.ss,
                                                      a.ss_np, a.kappa, i, j, cls, a.flags);
    if (lane == 0) store<KERNEL>(a.out, ee, v, a.flags);
  }
}

template <int KERNEL, int LAYER>
hipError_t launch_blocks_kl(bool coupling, const BlockArgs &a, hipStream_t s) {
  int tr, tc;
  size_t lds;
  block_tile_shape(a.nq_pad, LAYER, &tr, &tc, &lds);
  const int xc = rule_chunk(a.nq);
  const dim3 grid(a.nblocks), block(kThreads);
  const int cp = coupling ? 1 : 0;
  switch (xc) {
    case 4: hipLaunchKernelGGL((k_blocks<KERNEL, LAYER, 4>), grid, block, lds, s, a, cp); break;
    case 5: hipLaunchKernelGGL((k_blocks<KERNEL, LAYER, 5>), grid, block, lds, s, a, cp); break;
    case 7: hipLaunchKernelGGL((k_blocks<KERNEL, LAYER, 7>), grid, block, lds, s, a, cp); break;
    case 8: hipLaunchKernelGGL((k_blocks<KERNEL, LAYER, 8>), grid, block, lds, s, a, cp); break;
    default: hipLaunchKernelGGL((k_blocks<KERNEL, LAYER, 9>), grid, block, lds, s, a, cp); break;
  }
  return hipGetLastError();
}

}  // namespace

int rule_chunk(int nq) {
  for (int xc : {8, 9, 7, 5, 4})
    if (nq % xc == 0) return xc;
  return 4;
}

void block_tile_shape(int nq_pad, int layer, int *tr, int *tc, size_t *lds_bytes) {
  (void)layer;
  static const int shapes[][2] = {{64, 64}, {64, 32}, {64, 16}, {32, 16}, {16, 16},
                                  {16, 8},  {8, 8},   {8, 4},   {4, 4}};
  for (auto &sh : shapes) {
    const size_t dbl = (size_t)5 * nq_pad * sh[0] + (size_t)6 * nq_pad * sh[1] + 3 * sh[1];
    const size_t ints = (size_t)4 * sh[0] + 4 * sh[1] + (size_t)sh[0] * sh[1] + 2;
    const size_t bytes = dbl * 8 + ints * 4;
    *tr = sh[0];
    *tc = sh[1];
    *lds_bytes = bytes;
    if (bytes <= 64 * 1024) return;
  }
}

hipError_t launch_geometry(const bem_mesh &m, double *geo, int64_t ldg, unsigned *flags,
                           hipStream_t s) {
  if (m.nt == 0) return hipSuccess;
  hipLaunchKernelGGL(k_geometry, dim3((m.nt + 255) / 256), dim3(256), 0, s, m.v, m.nv, m.tri,
                     m.nt, geo, ldg, flags);
  return hipGetLastError();
}

hipError_t launch_blocks(int kernel, int layer, bool coupling, const BlockArgs &a, hipStream_t s) {
  if (a.nblocks == 0) return hipSuccess;
  if (kernel == BEM_LAPLACE)
    return layer == BEM_SLP ? launch_blocks_kl<BEM_LAPLACE, BEM_SLP>(coupling, a, s)
                            : launch_blocks_kl<BEM_LAPLACE, BEM_DLP>(coupling, a, s);
  return layer == BEM_SLP ? launch_blocks_kl<BEM_HELMHOLTZ, BEM_SLP>(coupling, a, s)
                          : launch_blocks_kl<BEM_HELMHOLTZ, BEM_DLP>(coupling, a, s);
}

hipError_t launch_entries(int kernel, int layer, const EntryArgs &a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const dim3 grid((unsigned)((a.n + kThreads - 1) / kThreads)), block(kThreads);
  if (kernel == BEM_LAPLACE) {
    if (layer == BEM_SLP) hipLaunchKernelGGL((k_entries<BEM_LAPLACE, BEM_SLP>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_entries<BEM_LAPLACE, BEM_DLP>), grid, block, 0, s, a);
  } else {
    if (layer == BEM_SLP) hipLaunchKernelGGL((k_entries<BEM_HELMHOLTZ, BEM_SLP>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_entries<BEM_HELMHOLTZ, BEM_DLP>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace bem
