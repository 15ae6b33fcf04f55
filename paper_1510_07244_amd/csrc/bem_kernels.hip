// HIP kernels for gfx950 (CDNA4, wave64): per-triangle geometry and the
// evaluation of arbitrary entry lists.  The block kernel is in bem_blocks.hip.
#include <hip/hip_runtime.h>

#include "bem_device.h"

namespace bem {
namespace {

using namespace dev;

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
    PairGeo g;
    if (pair_geometry(a.v, a.tri, a.nv, a.geo, a.ldg, i, j, cls, a.flags, &g)) {
      const Acc<KERNEL> v = ss_pair_wave<KERNEL, LAYER>(g, a.ss, cls, a.kappa);
      if (lane == 0) store<KERNEL>(a.out, ee, v, a.flags);
    }
  }
}

}  // namespace

hipError_t launch_geometry(const bem_mesh &m, double *geo, int64_t ldg, unsigned *flags,
                           hipStream_t s) {
  if (m.nt == 0) return hipSuccess;
  hipLaunchKernelGGL(k_geometry, dim3((m.nt + 255) / 256), dim3(256), 0, s, m.v, m.nv, m.tri,
                     m.nt, geo, ldg, flags);
  return hipGetLastError();
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
