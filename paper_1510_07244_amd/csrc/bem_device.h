// Device helpers shared by the kernels (gfx950, wave64): reciprocal square
// root, sine/cosine, accumulators, pair classification, the Sauter-Schwab
// relabelling and the wave-cooperative singular-pair quadrature.
#pragma once

#include <hip/hip_runtime.h>

#include "bem_internal.h"

namespace bem {
namespace dev {

constexpr double kInv4Pi = 0.0795774715459476678844418816863;  // 1 / (4 pi)
constexpr int kThreads = 256;
constexpr int kWave = 64;

// 1/sqrt(a) for a > 0: hardware estimate (relative error below 6e-8) and one
// Newton step y (3 - a y^2) / 2, which leaves a relative error near 1e-15.
__device__ __forceinline__ double rsqrt_newton(double a) {
  const double y = __builtin_amdgcn_rsq(a);
  const double t = a * y;
  const double e = fma(-t, y, 1.0);
  return fma(0.5 * y, e, y);
}

// sin and cos of x: Cody-Waite reduction x = k pi + r, |r| <= pi/2, with pi
// split into three parts (the first two with 33 significant bits so that
// k * part is exact for |k| < 2^20), then sin r = r + r^3 P(r^2) and
// cos r = 1 - r^2 / 2 + r^4 Q(r^2), P of degree 7 minimising the error
// relative to sin r and Q of degree 6 minimising the absolute error of cos r
// on [-pi/2, pi/2] (Remez exchange on the Taylor tail, computed by
// sincos_minimax.py beside this file: below 5.4e-18 relative and 1.4e-17
// absolute with the coefficients rounded to double); odd k negates both,
// by the sign bit.  Reducing by pi rather than pi/2 costs two more
// polynomial terms and saves the quadrant's exchange of sine and cosine.
constexpr double kOneOverPi = 0.31830988618379067154;
constexpr double kPia = 3.1415926534682512;      // 0x1.921fb544p+1
constexpr double kPib = 1.2154201012607932e-10;  // 0x1.0b4611a6p-33
constexpr double kPic = 4.044532497591901e-21;   // 0x1.3198a2e037073p-68

// x with its sign flipped when bit 31 of sgn is set
__device__ __forceinline__ double flip_sign(double x, int sgn) {
  return __hiloint2double(__double2hiint(x) ^ sgn, __double2loint(x));
}

__device__ __forceinline__ void sincos_cw(double x, double *s, double *c) {
  const double k = __builtin_rint(x * kOneOverPi);
  double r = fma(-k, kPia, x);
  r = fma(-k, kPib, r);
  r = fma(-k, kPic, r);
  const double r2 = r * r;
  double ps = 0x1.8829a2ffb2991p-49;  // P, highest degree first
  ps = fma(ps, r2, -0x1.ae431d98dda7bp-41);
  ps = fma(ps, r2, 0x1.6123cb29045c6p-33);
  ps = fma(ps, r2, -0x1.ae6454cb574e2p-26);
  ps = fma(ps, r2, 0x1.71de3a5287c76p-19);
  ps = fma(ps, r2, -0x1.a01a01a0148bcp-13);
  ps = fma(ps, r2, 0x1.11111111110c1p-7);
  ps = fma(ps, r2, -0x1.5555555555555p-3);
  const double sr = fma(r * r2, ps, r);
  double pc = 0x1.9fc8d3c9114a6p-45;  // Q, highest degree first
  pc = fma(pc, r2, -0x1.93573fa1f69b4p-37);
  pc = fma(pc, r2, 0x1.1eecfaec8e87dp-29);
  pc = fma(pc, r2, -0x1.27e4f9f33e2edp-22);
  pc = fma(pc, r2, 0x1.a01a019ba7403p-16);
  pc = fma(pc, r2, -0x1.6c16c16c10218p-10);
  pc = fma(pc, r2, 0x1.55555555554ddp-5);
  pc = fma(pc, r2, -0.5);
  const double cr = fma(r2, pc, 1.0);
  const int sgn = static_cast<int>((static_cast<unsigned>(static_cast<int>(k)) & 1u) << 31);
  *s = flip_sign(sr, sgn);
  *c = flip_sign(cr, sgn);
}

// FP32 sine and cosine for the mixed-precision path: the same reduction by
// pi, truncated to 12 + 12 + 24 significant bits (k * part exact for
// |k| < 2^12), minimax P and Q of degree 3 from the same construction (errors
// below 9.7e-9 relative and 5.8e-9 absolute with the coefficients rounded to
// float).
__device__ __forceinline__ void sincos_cw_f32(float x, float *s, float *c) {
  const float k = __builtin_rintf(x * 0.31830988f);
  float r = fmaf(-k, 3.140625f, x);               // 0x1.92p+1
  r = fmaf(-k, 9.67502593994140625e-4f, r);       // 0x1.fb4p-11
  r = fmaf(-k, 1.5099579e-7f, r);                 // 0x1.4442dp-23
  const float r2 = r * r;
  float ps = 0x1.5dbdf0p-19f;
  ps = fmaf(ps, r2, -0x1.9f6ffep-13f);
  ps = fmaf(ps, r2, 0x1.110ed4p-7f);
  ps = fmaf(ps, r2, -0x1.55554cp-3f);
  const float sr = fmaf(r * r2, ps, r);
  float pc = -0x1.194102p-22f;
  pc = fmaf(pc, r2, 0x1.9f8f5ap-16f);
  pc = fmaf(pc, r2, -0x1.6c149cp-10f);
  pc = fmaf(pc, r2, 0x1.555550p-5f);
  pc = fmaf(pc, r2, -0.5f);
  const float cr = fmaf(r2, pc, 1.0f);
  const int sgn = static_cast<int>((static_cast<unsigned>(static_cast<int>(k)) & 1u) << 31);
  *s = __int_as_float(__float_as_int(sr) ^ sgn);
  *c = __int_as_float(__float_as_int(cr) ^ sgn);
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
__device__ __forceinline__ void store(void *out, int64_t k, const Acc<KERNEL> &v,
                                      unsigned *flags) {
  if constexpr (KERNEL == BEM_LAPLACE) {
    if (!isfinite(v.re)) atomicOr(flags, FLAG_NONFINITE);
    static_cast<double *>(out)[k] = v.re;
  } else {
    if (!isfinite(v.re) || !isfinite(v.im)) atomicOr(flags, FLAG_NONFINITE);
    static_cast<double2 *>(out)[k] = make_double2(v.re, v.im);
  }
}

// Store for the plain (double / double2) or mixed (float / float2) output.
template <int KERNEL, bool MIXED>
__device__ __forceinline__ void store_as(void *out, int64_t k, const Acc<KERNEL> &v,
                                         unsigned *flags) {
  if constexpr (!MIXED) {
    store<KERNEL>(out, k, v, flags);
  } else if constexpr (KERNEL == BEM_LAPLACE) {
    const float r = static_cast<float>(v.re);
    if (!isfinite(r)) atomicOr(flags, FLAG_NONFINITE);
    static_cast<float *>(out)[k] = r;
  } else {
    const float r = static_cast<float>(v.re), i = static_cast<float>(v.im);
    if (!isfinite(r) || !isfinite(i)) atomicOr(flags, FLAG_NONFINITE);
    static_cast<float2 *>(out)[k] = make_float2(r, i);
  }
}

// One regular (disjoint) pair in FP64 with its rule points computed on the
// fly from the geometry arrays: sqrt(g_i g_j) sum_a w_a sum_b w_b k(x_a, y_b).
template <int KERNEL, int LAYER>
__device__ __forceinline__ Acc<KERNEL> regular_pair_fp64(const double *g, int64_t L,
                                                         const double *R, int nq, double kappa,
                                                         int i, int j) {
  double D[3], E1i[3], E2i[3], E1j[3], E2j[3];
  for (int c = 0; c < 3; ++c) {
    D[c] = g[(G_V0X + c) * L + i] - g[(G_V0X + c) * L + j];
    E1i[c] = g[(G_E1X + c) * L + i];
    E2i[c] = g[(G_E2X + c) * L + i];
    E1j[c] = g[(G_E1X + c) * L + j];
    E2j[c] = g[(G_E2X + c) * L + j];
  }
  const double nx = g[G_NX * L + j], ny = g[G_NY * L + j], nz = g[G_NZ * L + j];
  double are = 0.0, aim = 0.0;
  for (int qa = 0; qa < nq; ++qa) {
    double x[3];
    for (int c = 0; c < 3; ++c) x[c] = fma(R[qa], E1i[c], fma(R[nq + qa], E2i[c], D[c]));
    double ire = 0.0, iim = 0.0;
    for (int qb = 0; qb < nq; ++qb) {
      double d[3];
      for (int c = 0; c < 3; ++c) d[c] = fma(-R[qb], E1j[c], fma(-R[nq + qb], E2j[c], x[c]));
      const double r2 = fma(d[0], d[0], fma(d[1], d[1], d[2] * d[2]));
      const double z = rsqrt_newton(r2);
      double k = z;
      if constexpr (LAYER == BEM_DLP) k = fma(d[0], nx, fma(d[1], ny, d[2] * nz)) * z * z * z;
      const double w = R[2 * nq + qb];
      if constexpr (KERNEL == BEM_LAPLACE) {
        ire = fma(w, k, ire);
      } else {
        const double kr = kappa * r2 * z;
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
  return v;
}

__device__ __forceinline__ int shared_vertex_count(int a0, int a1, int a2, int b0, int b1, int b2) {
  return (a0 == b0) + (a0 == b1) + (a0 == b2) + (a1 == b0) + (a1 == b1) + (a1 == b2) +
         (a2 == b0) + (a2 == b1) + (a2 == b2);
}

// rotate (t0, t1, t2) left by k in {0, 1, 2}, without indexing an array
__device__ __forceinline__ void rotate3(int t0, int t1, int t2, int k, int *o0, int *o1, int *o2) {
  *o0 = k == 0 ? t0 : (k == 1 ? t1 : t2);
  *o1 = k == 0 ? t1 : (k == 1 ? t2 : t0);
  *o2 = k == 0 ? t2 : (k == 1 ? t0 : t1);
}

// Relabelling of a singular pair (common vertices first):
//   identical: mesh order; edge: the common vertices (lo, hi) by global id,
//   then the third vertex; vertex: the common vertex, then the other two in
//   the mesh's cyclic order.
__device__ __forceinline__ void relabel(int i0, int i1, int i2, int j0, int j1, int j2, int cls,
                                        int li[3], int lj[3]) {
  if (cls == CLS_IDENTICAL) {
    li[0] = i0, li[1] = i1, li[2] = i2;
    lj[0] = j0, lj[1] = j1, lj[2] = j2;
    return;
  }
  const bool s0 = i0 == j0 || i0 == j1 || i0 == j2;
  const bool s1 = i1 == j0 || i1 == j1 || i1 == j2;
  const bool s2 = i2 == j0 || i2 == j1 || i2 == j2;
  if (cls == CLS_EDGE) {
    const int ca = s0 ? i0 : i1;            // first common vertex in i's order
    const int cb = s2 ? i2 : (s1 && s0 ? i1 : i2);
    const int lo = min(ca, cb), hi = max(ca, cb);
    const int ci = !s0 ? i0 : (!s1 ? i1 : i2);
    const bool r0 = j0 == lo || j0 == hi, r1 = j1 == lo || j1 == hi;
    const int cj = !r0 ? j0 : (!r1 ? j1 : j2);
    li[0] = lo, li[1] = hi, li[2] = ci;
    lj[0] = lo, lj[1] = hi, lj[2] = cj;
    return;
  }
  const int ka = s0 ? 0 : (s1 ? 1 : 2);
  const int a = ka == 0 ? i0 : (ka == 1 ? i1 : i2);
  const int kb = j0 == a ? 0 : (j1 == a ? 1 : 2);
  rotate3(i0, i1, i2, ka, &li[0], &li[1], &li[2]);
  rotate3(j0, j1, j2, kb, &lj[0], &lj[1], &lj[2]);
}

// ---------------------------------------------------------- Sauter-Schwab
// After relabelling, both affine maps start at a common vertex, so for a rule
// point (x^, y^) = xi g(eta) the difference is x - y = xi d(eta) with
//   d = g1 E1_i + g2 E2_i - g3 E1_j - g4 E2_j,   r = xi |d|.
// With the Jacobian's factor xi^3 the xi sum of the Laplace kernels is a
// moment of the xi rule:  SLP  sum_a w_a xi_a^2 / |d|,
//                         DLP  sum_a w_a xi_a <d, n_j> / |d|^3;
// the Helmholtz kernels keep the xi sum (e^{i kappa xi |d|}).
struct PairGeo {
  double E1i[3], E2i[3], E1j[3], E2j[3], n[3];
  double scale;  // sqrt(g_i) sqrt(g_j) / (4 pi)
};

typedef const double __attribute__((address_space(4))) *uniform_ptr;

// Loads and relabels pair (i, j) of class cls; false (and the flag) if a
// vertex id is out of range.
__device__ __forceinline__ bool pair_geometry(const double *v, const int32_t *tri, int nv,
                                              const double *geo, int64_t ldg, int i, int j,
                                              int cls, unsigned *flags, PairGeo *g) {
  const int i0 = tri[3 * (int64_t)i], i1 = tri[3 * (int64_t)i + 1], i2 = tri[3 * (int64_t)i + 2];
  const int j0 = tri[3 * (int64_t)j], j1 = tri[3 * (int64_t)j + 1], j2 = tri[3 * (int64_t)j + 2];
  const bool ok = i0 >= 0 && i0 < nv && i1 >= 0 && i1 < nv && i2 >= 0 && i2 < nv && j0 >= 0 &&
                  j0 < nv && j1 >= 0 && j1 < nv && j2 >= 0 && j2 < nv;
  if (!ok) {
    atomicOr(flags, FLAG_EINVAL);
    return false;
  }
  int li[3], lj[3];
  relabel(i0, i1, i2, j0, j1, j2, cls, li, lj);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double pi0 = v[3 * (int64_t)li[0] + c], pi1 = v[3 * (int64_t)li[1] + c],
                 pi2 = v[3 * (int64_t)li[2] + c];
    const double pj0 = v[3 * (int64_t)lj[0] + c], pj1 = v[3 * (int64_t)lj[1] + c],
                 pj2 = v[3 * (int64_t)lj[2] + c];
    g->E1i[c] = pi1 - pi0;
    g->E2i[c] = pi2 - pi1;
    g->E1j[c] = pj1 - pj0;
    g->E2j[c] = pj2 - pj1;
  }
  g->n[0] = geo[G_NX * ldg + j];
  g->n[1] = geo[G_NY * ldg + j];
  g->n[2] = geo[G_NZ * ldg + j];
  g->scale = geo[G_SG * ldg + i] * geo[G_SG * ldg + j] * kInv4Pi;
  return true;
}

// Adds the contribution of one eta point (map g at xi = 1, eta weight w).
// Laplace sums are completed by the xi moment in ss_finish.
template <int KERNEL, int LAYER>
__device__ __forceinline__ void eta_point(const PairGeo &g, double g1, double g2, double g3,
                                          double g4, double w, const SSArgs &ss, double kappa,
                                          double *are, double *aim) {
  double d[3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
    d[c] = fma(g1, g.E1i[c], fma(g2, g.E2i[c], fma(-g3, g.E1j[c], -g4 * g.E2j[c])));
  const double rho2 = fma(d[0], d[0], fma(d[1], d[1], d[2] * d[2]));
  const double z = rsqrt_newton(rho2);  // 1 / |d|
  if constexpr (KERNEL == BEM_LAPLACE) {
    if constexpr (LAYER == BEM_SLP) {
      *are = fma(w, z, *are);
    } else {
      const double dn = fma(d[0], g.n[0], fma(d[1], g.n[1], d[2] * g.n[2]));
      *are = fma(w * dn, z * z * z, *are);
    }
  } else {
    const double rho = rho2 * z;
    const uniform_ptr X = (uniform_ptr)(ss.xi);
    const int q = ss.q;
    double base = w * z;  // SLP: w_a xi_a^2 e^{i k xi rho} / rho
    if constexpr (LAYER == BEM_DLP)
      base = w * fma(d[0], g.n[0], fma(d[1], g.n[1], d[2] * g.n[2])) * z * z * z;
    for (int a = 0; a < q; ++a) {
      const double xa = X[a];
      const double kr = kappa * xa * rho;
      double sn, cs;
      sincos_cw(kr, &sn, &cs);
      if constexpr (LAYER == BEM_SLP) {
        const double c = base * X[q + a];  // w_a xi_a^2
        *are = fma(c, cs, *are);
        *aim = fma(c, sn, *aim);
      } else {  // w_a xi_a e^{i kr} (1 - i kr) <d, n> / |d|^3
        const double c = base * X[2 * q + a];
        *are = fma(c, fma(kr, sn, cs), *are);
        *aim = fma(c, fma(-kr, cs, sn), *aim);
      }
    }
  }
}

template <int KERNEL, int LAYER>
__device__ __forceinline__ Acc<KERNEL> ss_finish(const PairGeo &g, const SSArgs &ss, double are,
                                                 double aim) {
  Acc<KERNEL> r;
  if constexpr (KERNEL == BEM_LAPLACE) {
    const uniform_ptr X = (uniform_ptr)(ss.xi);
    const double moment = LAYER == BEM_SLP ? X[3 * ss.q + 1] : X[3 * ss.q];
    r.re = are * moment * g.scale;
  } else {
    r.re = are * g.scale;
    r.im = aim * g.scale;
  }
  return r;
}

// One singular pair per lane; all lanes of the wave share the class, so the
// eta table is read with wave-uniform (scalar) loads.
// Table of a class for this kernel: identical pairs of a single layer use
// the symmetric half-table; for a double layer an identical pair's entry
// vanishes (on a flat triangle <x - y, n> = 0), so no point is summed.
template <int LAYER>
__device__ __forceinline__ int ss_table(int cls) {
  return cls == CLS_IDENTICAL && LAYER == BEM_SLP ? 0 : cls;
}
// Element k of a four-entry argument array by selects, not by an index: a
// kernel that copies its arguments into registers (the persistent form) would
// otherwise keep the whole copy in scratch memory.
template <class T>
__device__ __forceinline__ T pick4(const T (&v)[4], int k) {
  return k == 0 ? v[0] : k == 1 ? v[1] : k == 2 ? v[2] : v[3];
}
template <int LAYER>
__device__ __forceinline__ int ss_points(const SSArgs &ss, int cls) {
  return cls == CLS_IDENTICAL && LAYER == BEM_DLP ? 0 : pick4(ss.np, ss_table<LAYER>(cls));
}

template <int KERNEL, int LAYER>
__device__ __forceinline__ Acc<KERNEL> ss_pair_lane(const PairGeo &g, const SSArgs &ss, int cls,
                                                    double kappa) {
  const uniform_ptr T = (uniform_ptr)(pick4(ss.eta, ss_table<LAYER>(cls)));
  const int n = ss_points<LAYER>(ss, cls);
  // U eta points per step into U accumulators, written stage by stage so
  // that the independent chains interleave (the sum order is fixed)
  constexpr int U = KERNEL == BEM_LAPLACE ? 4 : 2;
  double are[U], aim[U];
#pragma unroll
  for (int u = 0; u < U; ++u) are[u] = 0.0, aim[u] = 0.0;
  int p = 0;
  if constexpr (KERNEL == BEM_LAPLACE) {
    for (; p + U <= n; p += U) {
      double d0[U], d1[U], d2[U], r2[U], h[U], w[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double g1 = T[p + u], g2 = T[n + p + u], g3 = T[2 * n + p + u], g4 = T[3 * n + p + u];
        w[u] = T[4 * n + p + u];
        d0[u] = fma(g1, g.E1i[0], fma(g2, g.E2i[0], fma(-g3, g.E1j[0], -g4 * g.E2j[0])));
        d1[u] = fma(g1, g.E1i[1], fma(g2, g.E2i[1], fma(-g3, g.E1j[1], -g4 * g.E2j[1])));
        d2[u] = fma(g1, g.E1i[2], fma(g2, g.E2i[2], fma(-g3, g.E1j[2], -g4 * g.E2j[2])));
      }
#pragma unroll
      for (int u = 0; u < U; ++u) r2[u] = fma(d0[u], d0[u], fma(d1[u], d1[u], d2[u] * d2[u]));
#pragma unroll
      for (int u = 0; u < U; ++u) h[u] = __builtin_amdgcn_rsq(r2[u]);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        // one Newton step: z = h + h (1 - r2 h^2) / 2 ~ 1 / |d|
        const double z = fma(0.5 * h[u], fma(-(r2[u] * h[u]), h[u], 1.0), h[u]);
        if constexpr (LAYER == BEM_SLP) {
          are[u] = fma(w[u], z, are[u]);
        } else {
          const double dn = fma(d0[u], g.n[0], fma(d1[u], g.n[1], d2[u] * g.n[2]));
          are[u] = fma(w[u] * dn, z * z * z, are[u]);
        }
      }
    }
  } else {
    for (; p + U <= n; p += U) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        eta_point<KERNEL, LAYER>(g, T[p + u], T[n + p + u], T[2 * n + p + u], T[3 * n + p + u],
                                 T[4 * n + p + u], ss, kappa, &are[u], &aim[u]);
    }
  }
  for (; p < n; ++p)
    eta_point<KERNEL, LAYER>(g, T[p], T[n + p], T[2 * n + p], T[3 * n + p], T[4 * n + p], ss,
                             kappa, &are[0], &aim[0]);
  double re = are[0], im = aim[0];
#pragma unroll
  for (int u = 1; u < U; ++u) re += are[u], im += aim[u];
  return ss_finish<KERNEL, LAYER>(g, ss, re, im);
}

// Both layers of one Helmholtz singular pair per lane in one pass over the
// eta points (edge- and vertex-adjacent pairs, whose single and double
// layer share the eta table): the difference vector, its length and the
// sine and cosine of every xi point serve both sums.  Each sum takes the
// same operands in the same order as ss_pair_lane's for its layer.
__device__ __forceinline__ void ss_pair_lane_both(const PairGeo &g, const SSArgs &ss, int cls,
                                                  double kappa, Acc<BEM_HELMHOLTZ> *vs,
                                                  Acc<BEM_HELMHOLTZ> *vd) {
  const uniform_ptr T = (uniform_ptr)(pick4(ss.eta, cls));
  const uniform_ptr X = (uniform_ptr)(ss.xi);
  const int n = pick4(ss.np, cls), q = ss.q;
  constexpr int U = 2;
  double sre[U], sim[U], dre[U], dim[U];
#pragma unroll
  for (int u = 0; u < U; ++u) sre[u] = sim[u] = dre[u] = dim[u] = 0.0;
  auto point = [&](int p, int u) {
    const double g1 = T[p], g2 = T[n + p], g3 = T[2 * n + p], g4 = T[3 * n + p];
    const double w = T[4 * n + p];
    double d[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      d[c] = fma(g1, g.E1i[c], fma(g2, g.E2i[c], fma(-g3, g.E1j[c], -g4 * g.E2j[c])));
    const double rho2 = fma(d[0], d[0], fma(d[1], d[1], d[2] * d[2]));
    const double z = rsqrt_newton(rho2);  // 1 / |d|
    const double rho = rho2 * z;
    const double bs = w * z;
    const double bd = w * fma(d[0], g.n[0], fma(d[1], g.n[1], d[2] * g.n[2])) * z * z * z;
    for (int a = 0; a < q; ++a) {
      const double xa = X[a];
      const double kr = kappa * xa * rho;
      double sn, cs;
      sincos_cw(kr, &sn, &cs);
      const double c1 = bs * X[q + a];  // w_a xi_a^2
      sre[u] = fma(c1, cs, sre[u]);
      sim[u] = fma(c1, sn, sim[u]);
      const double c2 = bd * X[2 * q + a];  // w_a xi_a
      dre[u] = fma(c2, fma(kr, sn, cs), dre[u]);
      dim[u] = fma(c2, fma(-kr, cs, sn), dim[u]);
    }
  };
  int p = 0;
  for (; p + U <= n; p += U) {
#pragma unroll
    for (int u = 0; u < U; ++u) point(p + u, u);
  }
  for (; p < n; ++p) point(p, 0);
  double a0 = sre[0], a1 = sim[0], b0 = dre[0], b1 = dim[0];
#pragma unroll
  for (int u = 1; u < U; ++u) a0 += sre[u], a1 += sim[u], b0 += dre[u], b1 += dim[u];
  *vs = ss_finish<BEM_HELMHOLTZ, BEM_SLP>(g, ss, a0, a1);
  *vd = ss_finish<BEM_HELMHOLTZ, BEM_DLP>(g, ss, b0, b1);
}

// One singular pair per wave: lanes stride over the eta points, then a
// butterfly sum.  Every lane returns the entry.
template <int KERNEL, int LAYER>
__device__ Acc<KERNEL> ss_pair_wave(const PairGeo &g, const SSArgs &ss, int cls, double kappa) {
  const int lane = threadIdx.x & (kWave - 1);
  const double *T = pick4(ss.eta, ss_table<LAYER>(cls));
  const int n = ss_points<LAYER>(ss, cls);
  double are = 0.0, aim = 0.0;
  for (int p = lane; p < n; p += kWave)
    eta_point<KERNEL, LAYER>(g, T[p], T[n + p], T[2 * n + p], T[3 * n + p], T[4 * n + p], ss,
                             kappa, &are, &aim);
  are = wave_sum(are);
  if constexpr (KERNEL == BEM_HELMHOLTZ) aim = wave_sum(aim);
  return ss_finish<KERNEL, LAYER>(g, ss, are, aim);
}

}  // namespace dev
}  // namespace bem
