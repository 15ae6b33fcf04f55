// Piecewise-linear (P1) bases (Sec. 2.2, eq. reference_integral: the
// transformed basis functions are low-order polynomials).  For a pair of
// triangles the 3 x 3 local matrix
//     L_ab = int_{tau_i} int_{tau_j} lambda_a(x) k(x, y) mu_b(y) dy dx
// (lambda_a, mu_b the nodal functions of the triangles' vertices in mesh
// order) comes from the same rules as the piecewise-constant entries: on
// the reference triangle of Phi(s, t) = v0 + s e1 + t e2 the barycentric
// coordinates are (1 - s, s - t, t), so every rule point adds its weighted
// kernel value times the nine products of shape-function values.  The
// Galerkin matrix of the vertices is then the sum of the local matrices over
// the triangles around each vertex pair (k_p1_gather, a fixed-order gather
// in place of a scatter-add, so results are reproducible bit for bit).
#include <hip/hip_runtime.h>

#include "bem_device.h"

namespace bem {
namespace {

using namespace dev;

// Nine sums in the pair's own vertex order (relabelled for singular pairs)
// and where each of its rows / columns goes in mesh order.
template <int KERNEL>
struct Acc9 {
  double re[9], im[9];
  int pr[3], pc[3];
};

// kernel value k(x, y) for d = x - y (r = |d|), n the normal of tau_j;
// Helmholtz as (re, im)
template <int KERNEL, int LAYER>
__device__ __forceinline__ void kernel_value(double dx, double dy, double dz, const double *n,
                                             double kappa, double *kre, double *kim) {
  const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
  const double iz = rsqrt_newton(r2);
  double base = iz;
  if constexpr (LAYER == BEM_DLP) base = fma(dx, n[0], fma(dy, n[1], dz * n[2])) * iz * iz * iz;
  if constexpr (KERNEL == BEM_LAPLACE) {
    *kre = base;
    *kim = 0.0;
  } else {
    const double kr = kappa * r2 * iz;
    double sn, cs;
    sincos_cw(kr, &sn, &cs);
    if constexpr (LAYER == BEM_SLP) {
      *kre = base * cs;
      *kim = base * sn;
    } else {  // e^{ikr} (1 - i kr)
      *kre = base * fma(kr, sn, cs);
      *kim = base * fma(-kr, cs, sn);
    }
  }
}

// Regular pair by the triangle rule of each triangle (lane per pair):
// inner sums over the column points for the three column shape functions,
// then the row point's three shape functions.
template <int KERNEL, int LAYER>
__device__ void p1_regular(const P1Args &a, int i, int j, Acc9<KERNEL> *L) {
  const int64_t G = a.ldg;
  const double *g = a.geo;
  double vi[3], e1i[3], e2i[3], vj[3], e1j[3], e2j[3], n[3];
  for (int c = 0; c < 3; ++c) {
    vi[c] = g[(G_V0X + c) * G + i], e1i[c] = g[(G_E1X + c) * G + i], e2i[c] = g[(G_E2X + c) * G + i];
    vj[c] = g[(G_V0X + c) * G + j], e1j[c] = g[(G_E1X + c) * G + j], e2j[c] = g[(G_E2X + c) * G + j];
    n[c] = g[(G_NX + c) * G + j];
  }
  for (int e = 0; e < 9; ++e) L->re[e] = L->im[e] = 0.0;
  for (int k = 0; k < 3; ++k) L->pr[k] = L->pc[k] = k;
  const int nq = a.nq;
  for (int p = 0; p < nq; ++p) {
    const double s = a.rule[p], t = a.rule[nq + p], w = a.rule[2 * nq + p];
    const double x0 = fma(s, e1i[0], fma(t, e2i[0], vi[0]));
    const double x1 = fma(s, e1i[1], fma(t, e2i[1], vi[1]));
    const double x2 = fma(s, e1i[2], fma(t, e2i[2], vi[2]));
    double ire[3] = {0, 0, 0}, iim[3] = {0, 0, 0};
    for (int q = 0; q < nq; ++q) {
      const double u = a.rule[q], v = a.rule[nq + q], wq = a.rule[2 * nq + q];
      const double y0 = fma(u, e1j[0], fma(v, e2j[0], vj[0]));
      const double y1 = fma(u, e1j[1], fma(v, e2j[1], vj[1]));
      const double y2 = fma(u, e1j[2], fma(v, e2j[2], vj[2]));
      double kre, kim;
      kernel_value<KERNEL, LAYER>(x0 - y0, x1 - y1, x2 - y2, n, a.kappa, &kre, &kim);
      const double mu[3] = {1.0 - u, u - v, v};
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        ire[b] = fma(wq * mu[b], kre, ire[b]);
        if constexpr (KERNEL == BEM_HELMHOLTZ) iim[b] = fma(wq * mu[b], kim, iim[b]);
      }
    }
    const double la[3] = {w * (1.0 - s), w * (s - t), w * t};
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        L->re[3 * k + b] = fma(la[k], ire[b], L->re[3 * k + b]);
        if constexpr (KERNEL == BEM_HELMHOLTZ) L->im[3 * k + b] = fma(la[k], iim[b], L->im[3 * k + b]);
      }
  }
  const double sc = g[G_SG * G + i] * g[G_SG * G + j] * kInv4Pi;
  for (int e = 0; e < 9; ++e) L->re[e] *= sc, L->im[e] *= sc;
}

// Singular pair by the Sauter-Schwab rule of its class (one wave per pair,
// lanes over the eta points; every xi node of the rule per eta point).
// After relabelling both maps start at a common vertex, so x - y = xi d(eta)
// with d = g1 E1_i + g2 E2_i - g3 E1_j - g4 E2_j; the shape functions are
// those of the relabelled vertices, summed into the mesh-order slots.
template <int KERNEL, int LAYER>
__device__ void p1_singular(const P1Args &a, int i, int j, int cls, Acc9<KERNEL> *L) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int e = 0; e < 9; ++e) L->re[e] = L->im[e] = 0.0;
  const int *ti = a.tri + 3 * (int64_t)i, *tj = a.tri + 3 * (int64_t)j;
  int li[3], lj[3];
  relabel(ti[0], ti[1], ti[2], tj[0], tj[1], tj[2], cls, li, lj);
  for (int k = 0; k < 3; ++k) {  // mesh-order slot of relabelled vertex k
    L->pr[k] = ti[0] == li[k] ? 0 : (ti[1] == li[k] ? 1 : 2);
    L->pc[k] = tj[0] == lj[k] ? 0 : (tj[1] == lj[k] ? 1 : 2);
  }
  PairGeo pg;
  if (!pair_geometry(a.v, a.tri, a.nv, a.geo, a.ldg, i, j, cls, a.flags, &pg)) return;
  if (!(LAYER == BEM_DLP && cls == CLS_IDENTICAL)) {  // else <x - y, n> = 0: all zero
    const double *T = pick4(a.ss.eta, cls);  // full tables (the identical one too)
    const int np = pick4(a.ss.np, cls), q = a.ss.q;
    const double *X = a.ss.xi;  // [xi | w xi^2 | w xi | ...]
    for (int p = lane; p < np; p += kWave) {
      const double g1 = T[p], g2 = T[np + p], g3 = T[2 * np + p], g4 = T[3 * np + p];
      const double wt = T[4 * np + p];
      double d[3];
#pragma unroll
      for (int c = 0; c < 3; ++c)
        d[c] = fma(g1, pg.E1i[c], fma(g2, pg.E2i[c], fma(-g3, pg.E1j[c], -g4 * pg.E2j[c])));
      for (int k = 0; k < q; ++k) {
        const double xi = X[k];
        const double w = wt * xi * X[q + k];  // eta weight x w_a xi_a^3
        double kre, kim;
        kernel_value<KERNEL, LAYER>(xi * d[0], xi * d[1], xi * d[2], pg.n, a.kappa, &kre, &kim);
        const double lx[3] = {1.0 - xi * g1, xi * (g1 - g2), xi * g2};
        const double ly[3] = {1.0 - xi * g3, xi * (g3 - g4), xi * g4};
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const int e = 3 * r + c;
            const double f = w * lx[r] * ly[c];
            L->re[e] = fma(f, kre, L->re[e]);
            if constexpr (KERNEL == BEM_HELMHOLTZ) L->im[e] = fma(f, kim, L->im[e]);
          }
      }
    }
  }
  for (int e = 0; e < 9; ++e) {
    L->re[e] = wave_sum(L->re[e]) * pg.scale;
    if constexpr (KERNEL == BEM_HELMHOLTZ) L->im[e] = wave_sum(L->im[e]) * pg.scale;
  }
}

template <int KERNEL>
__device__ __forceinline__ void store9(const P1Args &a, int64_t k, const Acc9<KERNEL> &L) {
  bool finite = true;
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    const int64_t dst = 9 * k + 3 * L.pr[e / 3] + L.pc[e % 3];
    if constexpr (KERNEL == BEM_LAPLACE) {
      static_cast<double *>(a.out)[dst] = L.re[e];
      finite = finite && isfinite(L.re[e]);
    } else {
      static_cast<double2 *>(a.out)[dst] = make_double2(L.re[e], L.im[e]);
      finite = finite && isfinite(L.re[e]) && isfinite(L.im[e]);
    }
  }
  if (!finite) atomicOr(a.flags, FLAG_NONFINITE);
}

template <int KERNEL, int LAYER>
__global__ __launch_bounds__(kThreads) void k_p1_pairs(const P1Args a) {
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
        Acc9<KERNEL> L;
        p1_regular<KERNEL, LAYER>(a, i, j, &L);
        store9<KERNEL>(a, e, L);
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
    Acc9<KERNEL> L;
    p1_singular<KERNEL, LAYER>(a, i, j, cls, &L);
    if (lane == 0) store9<KERNEL>(a, ee, L);
  }
}

// out[v + nrv w] = sum over (ta, ka) around row vertex v and (tb, kb) around
// column vertex w of local[(ta ntc + tb) 9 + 3 ka + kb], in list order.
template <bool CPLX>
__global__ __launch_bounds__(kThreads) void k_p1_gather(const P1GatherArgs a) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= (int64_t)a.nrv * a.ncv) return;
  const int v = (int)(e % a.nrv), w = (int)(e / a.nrv);
  const int r0 = a.rs_ptr[v], r1 = a.rs_ptr[v + 1], c0 = a.cs_ptr[w], c1 = a.cs_ptr[w + 1];
  if (r0 < 0 || r0 > r1 || r1 > a.rs_len || c0 < 0 || c0 > c1 || c1 > a.cs_len) {
    atomicOr(a.flags, FLAG_EINVAL);
    return;
  }
  double re = 0.0, im = 0.0;
  for (int p = r0; p < r1; ++p) {
    const int ta = a.rs_tri[p], ka = a.rs_loc[p];
    for (int q = c0; q < c1; ++q) {
      const int tb = a.cs_tri[q], kb = a.cs_loc[q];
      if (ta < 0 || ta >= a.ntr || tb < 0 || tb >= a.ntc || ka < 0 || ka > 2 || kb < 0 || kb > 2) {
        atomicOr(a.flags, FLAG_EINVAL);
        continue;
      }
      const int64_t k = ((int64_t)ta * a.ntc + tb) * 9 + 3 * ka + kb;
      if (CPLX) {
        re += static_cast<const double *>(a.local)[2 * k];
        im += static_cast<const double *>(a.local)[2 * k + 1];
      } else {
        re += static_cast<const double *>(a.local)[k];
      }
    }
  }
  if (CPLX) static_cast<double2 *>(a.out)[e] = make_double2(re, im);
  else static_cast<double *>(a.out)[e] = re;
}

}  // namespace

hipError_t launch_p1_pairs(int kernel, int layer, const P1Args &a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const dim3 grid((unsigned)((a.n + kThreads - 1) / kThreads)), block(kThreads);
  if (kernel == BEM_LAPLACE) {
    if (layer == BEM_SLP) hipLaunchKernelGGL((k_p1_pairs<BEM_LAPLACE, BEM_SLP>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_p1_pairs<BEM_LAPLACE, BEM_DLP>), grid, block, 0, s, a);
  } else {
    if (layer == BEM_SLP) hipLaunchKernelGGL((k_p1_pairs<BEM_HELMHOLTZ, BEM_SLP>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_p1_pairs<BEM_HELMHOLTZ, BEM_DLP>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_p1_gather(bool cplx, const P1GatherArgs &a, hipStream_t s) {
  const int64_t n = (int64_t)a.nrv * a.ncv;
  if (n == 0) return hipSuccess;
  const dim3 grid((unsigned)((n + kThreads - 1) / kThreads)), block(kThreads);
  if (cplx) hipLaunchKernelGGL(k_p1_gather<true>, grid, block, 0, s, a);
  else hipLaunchKernelGGL(k_p1_gather<false>, grid, block, 0, s, a);
  return hipGetLastError();
}

}  // namespace bem
