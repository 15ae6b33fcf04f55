// HIP kernels for gfx950 (CDNA4, wave64): per-triangle geometry and the
// evaluation of arbitrary entry lists.  The block kernel is in bem_blocks.hip.
#include <hip/hip_runtime.h>

#include <mutex>

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
// Arbitrary (i, j) list: one lane per regular entry (FP64, points computed on
// the fly); singular entries are listed and done by whole waves.  The mixed
// form stores the FP64 values rounded to FP32.
template <int KERNEL, int LAYER, bool MIXED>
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
        const Acc<KERNEL> v =
            regular_pair_fp64<KERNEL, LAYER>(a.geo, a.ldg, a.rule, a.nq, a.kappa, i, j);
        store_as<KERNEL, MIXED>(a.out, e, v, a.flags);
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
      if (lane == 0) store_as<KERNEL, MIXED>(a.out, ee, v, a.flags);
    }
  }
}

template <int KERNEL, int LAYER>
void launch_entries_kl(bool mixed, const EntryArgs &a, dim3 grid, dim3 block, hipStream_t s) {
  if (mixed) hipLaunchKernelGGL((k_entries<KERNEL, LAYER, true>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((k_entries<KERNEL, LAYER, false>), grid, block, 0, s, a);
}

// Fixed triangle-geometry scratch of the allocation-free near-field entry
// point: GEO_NF fields of up to BEM_NOALLOC_MAX_TRI triangles (leading
// dimension BEM_NOALLOC_MAX_TRI), one copy per GPU, held until the process
// ends.  Host code never passes this name to a kernel: it is a host-side
// stand-in; the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) double scratch[GEO_NF * (size_t)BEM_NOALLOC_MAX_TRI];

}  // namespace

hipError_t noalloc_scratch(int device, double **ptr) {
  // the array's address on each device, looked up once with that device
  // current (the caller makes it current) and kept
  static std::mutex mu;
  static double *addr[64] = {};
  if (device < 0 || device >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = static_cast<double *>(p);
  }
  *ptr = addr[device];
  return hipSuccess;
}

hipError_t launch_geometry(const bem_mesh &m, double *geo, int64_t ldg, unsigned *flags,
                           hipStream_t s) {
  if (m.nt == 0) return hipSuccess;
  hipLaunchKernelGGL(k_geometry, dim3((m.nt + 255) / 256), dim3(256), 0, s, m.v, m.nv, m.tri,
                     m.nt, geo, ldg, flags);
  return hipGetLastError();
}

hipError_t launch_entries(int kernel, int layer, bool mixed, const EntryArgs &a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const dim3 grid((unsigned)((a.n + kThreads - 1) / kThreads)), block(kThreads);
  if (kernel == BEM_LAPLACE) {
    if (layer == BEM_SLP) launch_entries_kl<BEM_LAPLACE, BEM_SLP>(mixed, a, grid, block, s);
    else launch_entries_kl<BEM_LAPLACE, BEM_DLP>(mixed, a, grid, block, s);
  } else {
    if (layer == BEM_SLP) launch_entries_kl<BEM_HELMHOLTZ, BEM_SLP>(mixed, a, grid, block, s);
    else launch_entries_kl<BEM_HELMHOLTZ, BEM_DLP>(mixed, a, grid, block, s);
  }
  return hipGetLastError();
}

}  // namespace bem
