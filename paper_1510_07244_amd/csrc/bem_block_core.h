// Building blocks of the block assembly kernels (gfx950, wave64): LDS layout
// of a sub-tile and the per-entry regular sums in FP64 and in FP32.  Shared by
// the per-block kernel and the persistent batched kernel (bem_blocks.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "bem_device.h"

namespace bem {
namespace blk {

using namespace dev;

constexpr double kPad = 1.0e4;       // coordinate of column padding points (weight 0)
constexpr uint16_t kNoPair = 0xffff; // empty slot of the sorted singular list
constexpr uint16_t kSwapped = 0x4000; // listed code: the mirror block's entry (j, i)
constexpr int kNearSingular = 0;     // list class of near-singular regular pairs (mixed)
constexpr int kSortPad = 512;        // room for the padding of up to 8 groups
constexpr int kBoth = 2;             // layer template value: single and double layer in one pass

// LDS layout of one sub-tile (up to TR rows x TC columns; triangle rule of nq
// points padded to nqp with zero weights):
//   ys[nqp][TC]    column points.  Plain: 6 doubles (-2Y0, -2Y1, -2Y2, |Y|^2,
//                  w sqrt(g_j), <Y, n_j>) with Y = 2 (y - c) in block-local
//                  coordinates.  Mixed: 8 floats (Y0, Y1, Y2, w sqrt(g_j),
//                  <Y, n_j>, pad) with Y = 2 (y - v0_j) local to the column
//                  triangle.  Read as 16-byte words (broadcast in a wave).
//   rg[10][TR]     row geometry 2 (v0 - c), 2 e1, 2 e2, sqrt(g_i)
//   rule[3][nqp]   s, t, w of the triangle rule
//   cn[3][TC]      column normals
//   both layers:   rn[3][TR] row normals
//   mixed only:    cg[3][TC] = 2 (v0_j - c); rb[6][TR], cb[6][TC] boxes
//   ints           rid[TR], rv[3][TR], cid[TC], cv[3][TC], count, bad,
//                  rcount, pad, per-group counts[16] and cursors[16]
//                  (classes at 0 .. 3, orders q at 8 + q)
//   list[TR*TC]    uint16 codes (row | col << 6 | group << 12, kSwapped) of the pairs
//                  left to the FP64 pass (singular; near-singular if mixed),
//                  from the front; with per-entry orders, the regular pairs
//                  (group = order) from the back
//   sorted[TR*TC + kSortPad]  codes grouped (by class or by order), each
//                  group padded to a multiple of 64 with kNoPair
struct Lds {
  double *ys, *rg, *rule, *cn, *rn, *cg, *rb, *cb;
  int *rid, *rv, *cid, *cv, *count, *bad, *rcount, *ccount, *cursor;
  uint16_t *list, *sorted;
};

__host__ __device__ __forceinline__ int ypoint_doubles(bool mixed) { return mixed ? 4 : 6; }

template <bool MIXED>
__device__ __forceinline__ Lds carve(double *base, int nqp, int TR, int TC, bool both = false) {
  Lds l;
  l.ys = base;
  l.rg = l.ys + ypoint_doubles(MIXED) * nqp * TC;
  l.rule = l.rg + 10 * TR;
  l.cn = l.rule + 3 * nqp;
  l.rn = both ? l.cn + 3 * TC : nullptr;
  l.cg = l.cn + 3 * TC + (both ? 3 * TR : 0);
  l.rb = l.cg + (MIXED ? 3 * TC : 0);
  l.cb = l.rb + (MIXED ? 6 * TR : 0);
  int *ib = reinterpret_cast<int *>(l.cb + (MIXED ? 6 * TC : 0));
  l.rid = ib;
  l.rv = l.rid + TR;
  l.cid = l.rv + 3 * TR;
  l.cv = l.cid + TC;
  l.count = l.cv + 3 * TC;
  l.bad = l.count + 1;
  l.rcount = l.bad + 1;
  l.ccount = l.rcount + 2;
  l.cursor = l.ccount + 16;
  l.list = reinterpret_cast<uint16_t *>(l.cursor + 16);
  l.sorted = l.list + TR * TC;
  return l;
}

// FP64 sum over the point pairs of one regular entry (sub-tile row rl,
// column cl): sum_b wy_b sum_a wx_a k'(x_a, y_b), where k' omits the factor
// 1/(4 pi) and, for the double layer, the factor 1/2 of the scaled normal
// distance.  4 |x - y|^2 = |X|^2 + |Y|^2 + X . (-2Y) in block-local
// coordinates; 1/r from v_rsq_f64 and one Newton step.  The double layer's
// wx <X - Y, n_j> is formed once per x-point (<Y, n_j> is constant on the
// column triangle's plane).
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
  // <Y, n_j> takes one value on the column triangle's plane: that of its
  // first point
  const double YN = LAYER == BEM_DLP ? ycol[2].y : 0.0;
  Acc<KERNEL> acc;
  for (int ch = 0; ch < nqp; ch += XC) {
    // WN = wx <X - Y, n_j>, the same for every column point
    double X0[XC], X1[XC], X2[XC], XX[XC], WX[XC], WN[XC];
#pragma unroll
    for (int a = 0; a < XC; ++a) {
      const double s = l.rule[ch + a], t = l.rule[nqp + ch + a], w = l.rule[2 * nqp + ch + a];
      X0[a] = fma(s, A0, fma(t, B0, D0));
      X1[a] = fma(s, A1, fma(t, B1, D1));
      X2[a] = fma(s, A2, fma(t, B2, D2));
      XX[a] = fma(X0[a], X0[a], fma(X1[a], X1[a], X2[a] * X2[a]));
      WX[a] = w * SG;
      if constexpr (LAYER == BEM_DLP)
        WN[a] = WX[a] * (fma(X0[a], n0, fma(X1[a], n1, X2[a] * n2)) - YN);
    }
    // one column point: (-2Y, |Y|^2, w sqrt(g_j), <Y, n_j>) as three double2
    auto point = [&](const double2 c0, const double2 c1, const double2 c2) {
      const double M0 = c0.x, M1 = c0.y, M2 = c1.x, YY = c1.y, WY = c2.x;
      // the XC chains are written stage by stage so that they interleave
      double sq[XC], h[XC];
#pragma unroll
      for (int a = 0; a < XC; ++a)
        sq[a] = fma(X2[a], M2, fma(X1[a], M1, fma(X0[a], M0, XX[a] + YY)));  // 4 r^2
#pragma unroll
      for (int a = 0; a < XC; ++a) h[a] = __builtin_amdgcn_rsq(sq[a]);     // ~ 1/(2r)
      double ire = 0.0, iim = 0.0;
#pragma unroll
      for (int a = 0; a < XC; ++a) {
        // one Newton step: z = h (3 - s h^2) ~ 1/r
        const double z = h[a] * fma(-(sq[a] * h[a]), h[a], 3.0);
        if constexpr (KERNEL == BEM_LAPLACE) {
          if constexpr (LAYER == BEM_SLP) {
            ire = fma(WX[a], z, ire);
          } else {
            ire = fma(WN[a], z * z * z, ire);  // wx 2 <x - y, n_j> / r^3
          }
        } else {
          const double kr = kq * sq[a] * z;  // kappa r  (kq = kappa / 4)
          double sn, cs;
          sincos_cw(kr, &sn, &cs);
          if constexpr (LAYER == BEM_SLP) {
            const double wz = WX[a] * z;
            ire = fma(wz, cs, ire);
            iim = fma(wz, sn, iim);
          } else {
            const double u = WN[a] * z * z * z;
            ire = fma(u, fma(kr, sn, cs), ire);
            iim = fma(u, fma(-kr, cs, sn), iim);
          }
        }
      }
      acc.re = fma(WY, ire, acc.re);
      if constexpr (KERNEL == BEM_HELMHOLTZ) acc.im = fma(WY, iim, acc.im);
    };
    // two points per step, the next one's LDS reads issued before the
    // current one's arithmetic (no register copies between steps)
    const double2 *yp = ycol;
    double2 a0 = yp[0], a1 = yp[1], a2 = yp[2];
    int kb = 0;
    for (; kb + 2 <= nqp; kb += 2) {
      const double2 *yn = yp + ystride;
      const double2 b0 = yn[0], b1 = yn[1], b2 = yn[2];
      __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the arithmetic
      point(a0, a1, a2);
      yp = ycol + (kb + 2 < nqp ? kb + 2 : nqp - 1) * ystride;
      a0 = yp[0], a1 = yp[1], a2 = yp[2];
      __builtin_amdgcn_sched_barrier(0);
      point(b0, b1, b2);
    }
    if (kb < nqp) point(a0, a1, a2);
  }
  return acc;
}

// One pass over the point pairs of regular entry (rl, cl) for both layers
// and for the double layer of the transposed pair (j, i), with k' as in
// regular_entry.  The distance, its reciprocal root (and for Helmholtz the
// sine and cosine) of a pair serve all three; with k3 the double layer's
// radial factor and, per column point b,
//   t1_b = sum_a wx_a k3_ab,   t2_b = sum_a wx_a <X_a - Y, n_j> k3_ab,
//   SLP(i, j) = sum_b wy_b sum_a wx_a k_ab,
//   DLP(i, j) = sum_b wy_b t2_b,
//   DLP(j, i) = sum_b wy_b (<Y_b, n_i> - <X, n_i>) t1_b,
// since <X_a, n_i> takes one value on the row triangle's plane and <Y_b, n_j>
// one on the column triangle's.  The point pairs of (j, i) are those of
// (i, j) with the roles of x and y exchanged: the same triangle rule on both.
template <int KERNEL, int XC>
__device__ __forceinline__ void regular_entry_both(const Lds &l, int TR, int TC, int nqp, int rl,
                                                   int cl, double kq, Acc<KERNEL> *gs,
                                                   Acc<KERNEL> *gd, Acc<KERNEL> *gm) {
  const double D0 = l.rg[0 * TR + rl], D1 = l.rg[1 * TR + rl], D2 = l.rg[2 * TR + rl];
  const double A0 = l.rg[3 * TR + rl], A1 = l.rg[4 * TR + rl], A2 = l.rg[5 * TR + rl];
  const double B0 = l.rg[6 * TR + rl], B1 = l.rg[7 * TR + rl], B2 = l.rg[8 * TR + rl];
  const double SG = l.rg[9 * TR + rl];
  const double n0 = l.cn[cl], n1 = l.cn[TC + cl], n2 = l.cn[2 * TC + cl];
  const double m0 = l.rn[rl], m1 = l.rn[TR + rl], m2 = l.rn[2 * TR + rl];
  const double XN = fma(D0, m0, fma(D1, m1, D2 * m2));  // <X, n_i>
  // -n_i / 2: <-2Y, -n_i / 2> = <Y, n_i>
  const double p0 = -0.5 * m0, p1 = -0.5 * m1, p2 = -0.5 * m2;
  const double2 *ycol = reinterpret_cast<const double2 *>(l.ys) + 3 * cl;
  const int ystride = 3 * TC;
  const double YN = ycol[2].y;  // <Y, n_j>: one value on the column triangle's plane
  Acc<KERNEL> s, d, m;
  for (int ch = 0; ch < nqp; ch += XC) {
    double X0[XC], X1[XC], X2[XC], XX[XC], WX[XC], WN[XC];
#pragma unroll
    for (int a = 0; a < XC; ++a) {
      const double u = l.rule[ch + a], t = l.rule[nqp + ch + a], w = l.rule[2 * nqp + ch + a];
      X0[a] = fma(u, A0, fma(t, B0, D0));
      X1[a] = fma(u, A1, fma(t, B1, D1));
      X2[a] = fma(u, A2, fma(t, B2, D2));
      XX[a] = fma(X0[a], X0[a], fma(X1[a], X1[a], X2[a] * X2[a]));
      WX[a] = w * SG;
      WN[a] = WX[a] * (fma(X0[a], n0, fma(X1[a], n1, X2[a] * n2)) - YN);  // wx <X - Y, n_j>
    }
    auto point = [&](const double2 c0, const double2 c1, const double2 c2) {
      const double M0 = c0.x, M1 = c0.y, M2 = c1.x, YY = c1.y, WY = c2.x;
      double sq[XC], h[XC];
#pragma unroll
      for (int a = 0; a < XC; ++a)
        sq[a] = fma(X2[a], M2, fma(X1[a], M1, fma(X0[a], M0, XX[a] + YY)));  // 4 r^2
#pragma unroll
      for (int a = 0; a < XC; ++a) h[a] = __builtin_amdgcn_rsq(sq[a]);
      double sre = 0.0, sim = 0.0, t1r = 0.0, t1i = 0.0, t2r = 0.0, t2i = 0.0;
#pragma unroll
      for (int a = 0; a < XC; ++a) {
        const double z = h[a] * fma(-(sq[a] * h[a]), h[a], 3.0);  // ~ 1/r
        const double z3 = z * z * z;
        if constexpr (KERNEL == BEM_LAPLACE) {
          sre = fma(WX[a], z, sre);
          t1r = fma(WX[a], z3, t1r);
          t2r = fma(WN[a], z3, t2r);
        } else {
          const double kr = kq * sq[a] * z;
          double sn, cs;
          sincos_cw(kr, &sn, &cs);
          const double wz = WX[a] * z;
          sre = fma(wz, cs, sre);
          sim = fma(wz, sn, sim);
          const double fr = z3 * fma(kr, sn, cs), fi = z3 * fma(-kr, cs, sn);
          t1r = fma(WX[a], fr, t1r);
          t1i = fma(WX[a], fi, t1i);
          t2r = fma(WN[a], fr, t2r);
          t2i = fma(WN[a], fi, t2i);
        }
      }
      const double wm = WY * (fma(M0, p0, fma(M1, p1, M2 * p2)) - XN);  // wy 2 <y - x, n_i>
      s.re = fma(WY, sre, s.re);
      d.re = fma(WY, t2r, d.re);
      m.re = fma(wm, t1r, m.re);
      if constexpr (KERNEL == BEM_HELMHOLTZ) {
        s.im = fma(WY, sim, s.im);
        d.im = fma(WY, t2i, d.im);
        m.im = fma(wm, t1i, m.im);
      }
    };
    const double2 *yp = ycol;
    double2 a0 = yp[0], a1 = yp[1], a2 = yp[2];
    int kb = 0;
    for (; kb + 2 <= nqp; kb += 2) {
      const double2 *yn = yp + ystride;
      const double2 b0 = yn[0], b1 = yn[1], b2 = yn[2];
      __builtin_amdgcn_sched_barrier(0);
      point(a0, a1, a2);
      yp = ycol + (kb + 2 < nqp ? kb + 2 : nqp - 1) * ystride;
      a0 = yp[0], a1 = yp[1], a2 = yp[2];
      __builtin_amdgcn_sched_barrier(0);
      point(b0, b1, b2);
    }
    if (kb < nqp) point(a0, a1, a2);
  }
  *gs = s;
  *gd = d;
  *gm = m;
}

// FP32 sum of one regular entry of the mixed form, in coordinates local to
// the row triangle's first vertex v0_i (per entry, so that the FP32 rounding
// of coordinates is relative to the pair's own size):
//   X_a = 2 (x_a - v0_i),  Y'_b = D + Y_b,  D = 2 (v0_j - v0_i) rounded once,
//   4 r^2 = |X|^2 + |Y'|^2 - 2 X . Y',  h = v_rsq_f32(4 r^2) = 1/(2r).
// Returns the same sum as regular_entry (with k' as there).
template <int KERNEL, int LAYER, int XC>
__device__ __forceinline__ Acc<KERNEL> regular_entry_f32(const Lds &l, int TR, int TC, int nqp,
                                                         int rl, int cl, double kappa) {
  const double A0 = l.rg[3 * TR + rl], A1 = l.rg[4 * TR + rl], A2 = l.rg[5 * TR + rl];
  const double B0 = l.rg[6 * TR + rl], B1 = l.rg[7 * TR + rl], B2 = l.rg[8 * TR + rl];
  const double SG = l.rg[9 * TR + rl];
  const float d0 = (float)(l.cg[cl] - l.rg[0 * TR + rl]);
  const float d1 = (float)(l.cg[TC + cl] - l.rg[1 * TR + rl]);
  const float d2 = (float)(l.cg[2 * TC + cl] - l.rg[2 * TR + rl]);
  float n0 = 0, n1 = 0, n2 = 0, dn = 0;
  if constexpr (LAYER == BEM_DLP) {
    n0 = (float)l.cn[cl];
    n1 = (float)l.cn[TC + cl];
    n2 = (float)l.cn[2 * TC + cl];
    dn = fmaf(d0, n0, fmaf(d1, n1, d2 * n2));
  }
  const float hk = 0.5f * (float)kappa;  // kappa r = (kappa / 2) (4 r^2) h
  const float4 *ycol = reinterpret_cast<const float4 *>(l.ys) + 2 * cl;
  const int ystride = 2 * TC;  // float4 per point index
  float are = 0.0f, aim = 0.0f;
  for (int ch = 0; ch < nqp; ch += XC) {
    // WN = wx <X - Y', n_j> = wx (<X, n_j> - <D, n_j>): <Y_b, n_j> vanishes on
    // the column triangle's plane
    float X0[XC], X1[XC], X2[XC], XX[XC], WX[XC], WN[XC];
#pragma unroll
    for (int a = 0; a < XC; ++a) {
      const double s = l.rule[ch + a], t = l.rule[nqp + ch + a], w = l.rule[2 * nqp + ch + a];
      const float x0 = (float)fma(s, A0, t * B0), x1 = (float)fma(s, A1, t * B1),
                  x2 = (float)fma(s, A2, t * B2);
      XX[a] = fmaf(x0, x0, fmaf(x1, x1, x2 * x2));
      X0[a] = -2.0f * x0;
      X1[a] = -2.0f * x1;
      X2[a] = -2.0f * x2;
      // h = 1/(2r): the SLP's k' = 1/r = 2h, the DLP's k' = 2 <x - y, n> / r^3
      // = 8 h^3 <X - Y', n> (same k' as the FP64 path)
      WX[a] = (float)(w * SG) * (LAYER == BEM_SLP ? 2.0f : 8.0f);
      if constexpr (LAYER == BEM_DLP) WN[a] = WX[a] * (fmaf(x0, n0, fmaf(x1, n1, x2 * n2)) - dn);
    }
    // one column point: (Y, w sqrt(g_j), <Y, n_j>) as two float4
    auto point = [&](const float4 c0, const float4 c1) {
      const float y0 = d0 + c0.x, y1 = d1 + c0.y, y2 = d2 + c0.z, WY = c0.w;
      const float YY = fmaf(y0, y0, fmaf(y1, y1, y2 * y2));
      // the XC chains are written stage by stage so that they interleave
      float sq[XC], h[XC];
#pragma unroll
      for (int a = 0; a < XC; ++a)
        sq[a] = fmaf(X2[a], y2, fmaf(X1[a], y1, fmaf(X0[a], y0, XX[a] + YY)));  // 4 r^2
#pragma unroll
      for (int a = 0; a < XC; ++a) h[a] = __builtin_amdgcn_rsqf(sq[a]);
      float ire = 0.0f, iim = 0.0f;
#pragma unroll
      for (int a = 0; a < XC; ++a) {
        if constexpr (KERNEL == BEM_LAPLACE) {
          if constexpr (LAYER == BEM_SLP) {
            ire = fmaf(WX[a], h[a], ire);
          } else {
            ire = fmaf(WN[a], h[a] * h[a] * h[a], ire);
          }
        } else {
          const float kr = hk * sq[a] * h[a];
          float sn, cs;
          sincos_cw_f32(kr, &sn, &cs);
          if constexpr (LAYER == BEM_SLP) {
            const float wz = WX[a] * h[a];
            ire = fmaf(wz, cs, ire);
            iim = fmaf(wz, sn, iim);
          } else {
            const float u = WN[a] * h[a] * h[a] * h[a];
            ire = fmaf(u, fmaf(kr, sn, cs), ire);
            iim = fmaf(u, fmaf(-kr, cs, sn), iim);
          }
        }
      }
      are = fmaf(WY, ire, are);
      if constexpr (KERNEL == BEM_HELMHOLTZ) aim = fmaf(WY, iim, aim);
    };
    // two points per step, the next one's LDS reads issued first
    const float4 *yp = ycol;
    float4 a0 = yp[0], a1 = yp[1];
    int kb = 0;
    for (; kb + 2 <= nqp; kb += 2) {
      const float4 *yn = yp + ystride;
      const float4 b0 = yn[0], b1 = yn[1];
      __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the arithmetic
      point(a0, a1);
      yp = ycol + (kb + 2 < nqp ? kb + 2 : nqp - 1) * ystride;
      a0 = yp[0], a1 = yp[1];
      __builtin_amdgcn_sched_barrier(0);
      point(b0, b1);
    }
    if (kb < nqp) point(a0, a1);
  }
  Acc<KERNEL> acc;
  acc.re = are;
  if constexpr (KERNEL == BEM_HELMHOLTZ) acc.im = aim;
  return acc;
}

// The one-pass form of regular_entry_f32 (see regular_entry_both): both
// layers of entry (rl, cl) and the double layer of the pair (j, i), in
// coordinates local to the row triangle's first vertex, where <X, n_i> = 0
// for every x-point, so that DLP(j, i) = sum_b wy_b <Y'_b, n_i> t1_b.
// h = v_rsq_f32(4 r^2) = 1/(2r): the single layer's k' = 2h, the double
// layer's radial factor 8 h^3 (the factors 2 and 8 are applied to the sums).
template <int KERNEL, int XC>
__device__ __forceinline__ void regular_entry_both_f32(const Lds &l, int TR, int TC, int nqp,
                                                       int rl, int cl, double kappa,
                                                       Acc<KERNEL> *gs, Acc<KERNEL> *gd,
                                                       Acc<KERNEL> *gm) {
  const double A0 = l.rg[3 * TR + rl], A1 = l.rg[4 * TR + rl], A2 = l.rg[5 * TR + rl];
  const double B0 = l.rg[6 * TR + rl], B1 = l.rg[7 * TR + rl], B2 = l.rg[8 * TR + rl];
  const double SG = l.rg[9 * TR + rl];
  const float d0 = (float)(l.cg[cl] - l.rg[0 * TR + rl]);
  const float d1 = (float)(l.cg[TC + cl] - l.rg[1 * TR + rl]);
  const float d2 = (float)(l.cg[2 * TC + cl] - l.rg[2 * TR + rl]);
  const float n0 = (float)l.cn[cl], n1 = (float)l.cn[TC + cl], n2 = (float)l.cn[2 * TC + cl];
  const float m0 = (float)l.rn[rl], m1 = (float)l.rn[TR + rl], m2 = (float)l.rn[2 * TR + rl];
  const float dn = fmaf(d0, n0, fmaf(d1, n1, d2 * n2));  // <D, n_j>
  const float hk = 0.5f * (float)kappa;
  const float4 *ycol = reinterpret_cast<const float4 *>(l.ys) + 2 * cl;
  const int ystride = 2 * TC;
  float sre = 0.0f, sim = 0.0f, dre = 0.0f, dim = 0.0f, mre = 0.0f, mim = 0.0f;
  for (int ch = 0; ch < nqp; ch += XC) {
    float X0[XC], X1[XC], X2[XC], XX[XC], WX[XC], WN[XC];
#pragma unroll
    for (int a = 0; a < XC; ++a) {
      const double u = l.rule[ch + a], t = l.rule[nqp + ch + a], w = l.rule[2 * nqp + ch + a];
      const float x0 = (float)fma(u, A0, t * B0), x1 = (float)fma(u, A1, t * B1),
                  x2 = (float)fma(u, A2, t * B2);
      XX[a] = fmaf(x0, x0, fmaf(x1, x1, x2 * x2));
      X0[a] = -2.0f * x0;
      X1[a] = -2.0f * x1;
      X2[a] = -2.0f * x2;
      WX[a] = (float)(w * SG);
      WN[a] = WX[a] * (fmaf(x0, n0, fmaf(x1, n1, x2 * n2)) - dn);  // wx <X - Y', n_j>
    }
    auto point = [&](const float4 c0) {
      const float y0 = d0 + c0.x, y1 = d1 + c0.y, y2 = d2 + c0.z, WY = c0.w;
      const float YY = fmaf(y0, y0, fmaf(y1, y1, y2 * y2));
      float sq[XC], h[XC];
#pragma unroll
      for (int a = 0; a < XC; ++a)
        sq[a] = fmaf(X2[a], y2, fmaf(X1[a], y1, fmaf(X0[a], y0, XX[a] + YY)));  // 4 r^2
#pragma unroll
      for (int a = 0; a < XC; ++a) h[a] = __builtin_amdgcn_rsqf(sq[a]);
      float tsr = 0.0f, tsi = 0.0f, t1r = 0.0f, t1i = 0.0f, t2r = 0.0f, t2i = 0.0f;
#pragma unroll
      for (int a = 0; a < XC; ++a) {
        const float h3 = h[a] * h[a] * h[a];
        if constexpr (KERNEL == BEM_LAPLACE) {
          tsr = fmaf(WX[a], h[a], tsr);
          t1r = fmaf(WX[a], h3, t1r);
          t2r = fmaf(WN[a], h3, t2r);
        } else {
          const float kr = hk * sq[a] * h[a];
          float sn, cs;
          sincos_cw_f32(kr, &sn, &cs);
          const float wz = WX[a] * h[a];
          tsr = fmaf(wz, cs, tsr);
          tsi = fmaf(wz, sn, tsi);
          const float fr = h3 * fmaf(kr, sn, cs), fi = h3 * fmaf(-kr, cs, sn);
          t1r = fmaf(WX[a], fr, t1r);
          t1i = fmaf(WX[a], fi, t1i);
          t2r = fmaf(WN[a], fr, t2r);
          t2i = fmaf(WN[a], fi, t2i);
        }
      }
      const float wm = WY * fmaf(y0, m0, fmaf(y1, m1, y2 * m2));  // wy <Y', n_i>
      sre = fmaf(WY, tsr, sre);
      dre = fmaf(WY, t2r, dre);
      mre = fmaf(wm, t1r, mre);
      if constexpr (KERNEL == BEM_HELMHOLTZ) {
        sim = fmaf(WY, tsi, sim);
        dim = fmaf(WY, t2i, dim);
        mim = fmaf(wm, t1i, mim);
      }
    };
    const float4 *yp = ycol;
    float4 a0 = yp[0];
    int kb = 0;
    for (; kb + 2 <= nqp; kb += 2) {
      const float4 b0 = (yp + ystride)[0];
      __builtin_amdgcn_sched_barrier(0);
      point(a0);
      yp = ycol + (kb + 2 < nqp ? kb + 2 : nqp - 1) * ystride;
      a0 = yp[0];
      __builtin_amdgcn_sched_barrier(0);
      point(b0);
    }
    if (kb < nqp) point(a0);
  }
  // k' factors: 2 for the single layer, 8 for the double layer
  gs->re = 2.0 * sre;
  gd->re = 8.0 * dre;
  gm->re = 8.0 * mre;
  if constexpr (KERNEL == BEM_HELMHOLTZ) {
    gs->im = 2.0 * sim;
    gd->im = 8.0 * dim;
    gm->im = 8.0 * mim;
  }
}

}  // namespace blk
}  // namespace bem
