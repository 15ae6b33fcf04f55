// Matrix-vector kernels of the H^2 matrix (Sec. 2.3-2.4: near-field blocks,
// nested cluster bases, coupling matrices) and the vector operations of the
// iterative solvers that use it (Sec. 4: conjugate gradients for the Laplace
// single layer; the Brakhage-Werner system for Helmholtz).
//
// The product is a handful of grouped, gathered small matrix-vector products
// (forward transformation of the column basis, coupling, backward
// transformation of the row basis, near field).  Each reads its matrices
// once, so it is bound by HBM bandwidth, not arithmetic: the kernels read
// every matrix column-wise with 64 consecutive lanes on 64 consecutive rows
// (one 512-byte line per wave and column) and keep the gathered input in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "bem_device.h"

namespace bem {
namespace {

using namespace dev;

constexpr int kMaxVec = 512;  // longest output and input of one group / block
constexpr int kChunks = kMaxVec / kWave;

template <bool CPLX>
struct Num;
template <>
struct Num<false> {
  double v;
  __device__ static Num zero() { Num r; r.v = 0.0; return r; }
  __device__ void fma_into(const double *A, int64_t k, const Num &x) { v = fma(A[k], x.v, v); }
  __device__ static Num load(const double *p, int64_t k) { Num r; r.v = p[k]; return r; }
  __device__ void add_to(double *p, int64_t k) const { p[k] += v; }
  __device__ void add(const Num &o) { v += o.v; }
  __device__ Num shfl_down_sum() const {
    Num r = *this;
    for (int o = kWave / 2; o >= 1; o >>= 1) r.v += __shfl_xor(r.v, o, kWave);
    return r;
  }
};
template <>
struct Num<true> {
  double re, im;
  __device__ static Num zero() { Num r; r.re = r.im = 0.0; return r; }
  __device__ void fma_into(const double *A, int64_t k, const Num &x) {
    const double ar = A[2 * k], ai = A[2 * k + 1];
    re = fma(ar, x.re, re);
    re = fma(-ai, x.im, re);
    im = fma(ar, x.im, im);
    im = fma(ai, x.re, im);
  }
  __device__ static Num load(const double *p, int64_t k) {
    Num r;
    r.re = p[2 * k];
    r.im = p[2 * k + 1];
    return r;
  }
  __device__ void add_to(double *p, int64_t k) const {
    p[2 * k] += re;
    p[2 * k + 1] += im;
  }
  __device__ void add(const Num &o) { re += o.re, im += o.im; }
  __device__ Num shfl_down_sum() const {
    Num r = *this;
    for (int o = kWave / 2; o >= 1; o >>= 1) {
      r.re += __shfl_xor(r.re, o, kWave);
      r.im += __shfl_xor(r.im, o, kWave);
    }
    return r;
  }
};

// Group g: y[out_idx[out_ptr[g] ..]] += sum_{b in group g} op(A_b) x[in_idx[in_ptr[b] ..]],
// op(A) = A (TRANS false; A is m_out x n_in) or A^T (TRANS true; A is
// n_in x m_out), column-major with the row count as leading dimension.  One
// workgroup per group; the sum over a group's blocks and inside each block
// runs in a fixed order (results are reproducible bit for bit).
template <bool CPLX, bool TRANS>
__global__ __launch_bounds__(kThreads) void k_gemv(const GemvArgs a) {
  using T = Num<CPLX>;
  __shared__ T xs[kMaxVec];
  __shared__ T part[kThreads / kWave][kMaxVec];
  __shared__ int bad;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  constexpr int W = kThreads / kWave;
  const double *A = static_cast<const double *>(a.A);
  const double *x = static_cast<const double *>(a.x);
  double *y = static_cast<double *>(a.y);
  for (int g = blockIdx.x; g < a.ngroups; g += gridDim.x) {
    const int64_t o0 = a.out_ptr[g], o1 = a.out_ptr[g + 1];
    const int64_t b0 = a.grp_ptr[g], b1 = a.grp_ptr[g + 1];
    const int64_t m = o1 - o0;
    if (!(o0 >= 0 && o0 <= o1 && o1 <= a.out_len && m <= kMaxVec && b0 >= 0 && b0 <= b1 &&
          b1 <= a.nblocks)) {
      if (tid == 0) atomicOr(a.flags, FLAG_EINVAL);
      continue;  // uniform
    }
    T acc[kChunks];  // TRANS false: rows lane + 64 c of this wave's columns
    for (int i = tid; i < W * kMaxVec; i += kThreads) part[i / kMaxVec][i % kMaxVec] = T::zero();
    __syncthreads();
    for (int64_t b = b0; b < b1; ++b) {
      const int64_t i0 = a.in_ptr[b], i1 = a.in_ptr[b + 1];
      const int64_t n = i1 - i0;
      const int64_t off = a.a_off[b];
      __syncthreads();  // xs of the previous block no longer read
      if (tid == 0) bad = !(i0 >= 0 && i0 <= i1 && i1 <= a.in_len && n <= kMaxVec && off >= 0 &&
                            off <= a.a_len && (m == 0 || n <= (a.a_len - off) / m));
      __syncthreads();
      if (bad) {
        if (tid == 0) atomicOr(a.flags, FLAG_EINVAL);
        continue;  // uniform
      }
      for (int64_t k = tid; k < n; k += kThreads) {
        const int id = a.in_idx[i0 + k];
        if (id < 0 || id >= a.x_len) {
          atomicOr(a.flags, FLAG_EINVAL);
          xs[k] = T::zero();
        } else {
          xs[k] = T::load(x, id);
        }
      }
      __syncthreads();
      if (!TRANS) {
        // wave w takes the columns j = w, w + 4, ...; lane l the rows l + 64 c
        for (int c = 0; c < kChunks; ++c) acc[c] = T::zero();
        for (int64_t j = wave; j < n; j += W) {
          const T xj = xs[j];
#pragma unroll
          for (int c = 0; c < kChunks; ++c) {
            const int64_t i = lane + kWave * c;
            if (i < m) acc[c].fma_into(A, off + i + m * j, xj);
          }
        }
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
          const int64_t i = lane + kWave * c;
          if (i < m) part[wave][i].add(acc[c]);
        }
      } else {
        // wave w takes the outputs j = w, w + 4, ...; lanes run down column j
        for (int64_t j = wave; j < m; j += W) {
          T s = T::zero();
          for (int64_t i = lane; i < n; i += kWave) s.fma_into(A, off + i + n * j, xs[i]);
          s = s.shfl_down_sum();
          if (lane == 0) part[wave][j].add(s);
        }
      }
    }
    __syncthreads();
    for (int64_t k = tid; k < m; k += kThreads) {
      T s = part[0][k];
      for (int w = 1; w < W; ++w) s.add(part[w][k]);
      const int id = a.out_idx[o0 + k];
      if (id < 0 || id >= a.y_len) atomicOr(a.flags, FLAG_EINVAL);
      else s.add_to(y, id);
    }
    __syncthreads();  // part is cleared for the next group
  }
}

// ------------------------------------------------------------ vector ops
constexpr int kDotBlocks = 256;

// Partial sums of sum_i conj?(x_i) y_i: workgroup b takes the fixed strided
// set of indices b * 256 + t + 256 * 256 * r, reduced in a fixed order.
template <bool CPLX, bool CONJ>
__global__ __launch_bounds__(kThreads) void k_dot_part(int64_t n, const double *x, const double *y,
                                                       double *part) {
  __shared__ double sr[kThreads], si[kThreads];
  double re = 0.0, im = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    if (CPLX) {
      const double xr = x[2 * i], xi = CONJ ? -x[2 * i + 1] : x[2 * i + 1];
      const double yr = y[2 * i], yi = y[2 * i + 1];
      re = fma(xr, yr, re);
      re = fma(-xi, yi, re);
      im = fma(xr, yi, im);
      im = fma(xi, yr, im);
    } else {
      re = fma(x[i], y[i], re);
    }
  }
  sr[threadIdx.x] = re;
  si[threadIdx.x] = im;
  __syncthreads();
  for (int s = kThreads / 2; s >= 1; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      si[threadIdx.x] += si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sr[0];
    part[2 * blockIdx.x + 1] = si[0];
  }
}

__global__ __launch_bounds__(kThreads) void k_dot_final(int nparts, const double *part,
                                                        double *out) {
  __shared__ double sr[kThreads], si[kThreads];
  double re = 0.0, im = 0.0;
  for (int k = threadIdx.x; k < nparts; k += kThreads) re += part[2 * k], im += part[2 * k + 1];
  sr[threadIdx.x] = re;
  si[threadIdx.x] = im;
  __syncthreads();
  for (int s = kThreads / 2; s >= 1; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      si[threadIdx.x] += si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sr[0], out[1] = si[0];
}

// y = alpha x + beta y (complex alpha, beta; real vectors use the real parts)
template <bool CPLX>
__global__ __launch_bounds__(kThreads) void k_axpby(int64_t n, double ar, double ai,
                                                    const double *x, double br, double bi,
                                                    double *y) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    if (CPLX) {
      const double xr = x[2 * i], xi = x[2 * i + 1], yr = y[2 * i], yi = y[2 * i + 1];
      y[2 * i] = ar * xr - ai * xi + (br * yr - bi * yi);
      y[2 * i + 1] = ar * xi + ai * xr + (br * yi + bi * yr);
    } else {
      y[i] = ar * x[i] + br * y[i];
    }
  }
}

// y += c M x, M the Galerkin mass matrix of piecewise constants: diagonal,
// M_ii = |tau_i| = sqrt(g_i) / 2
template <bool CPLX>
__global__ __launch_bounds__(kThreads) void k_mass(int32_t nt, const double *geo, int64_t ldg,
                                                   double cr, double ci, const double *x,
                                                   double *y) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= nt) return;
  const double area = 0.5 * geo[G_SG * ldg + i];
  if (CPLX) {
    const double xr = x[2 * i], xi = x[2 * i + 1];
    y[2 * i] += area * (cr * xr - ci * xi);
    y[2 * i + 1] += area * (cr * xi + ci * xr);
  } else {
    y[i] += area * cr * x[i];
  }
}

}  // namespace

hipError_t launch_gemv(bool cplx, bool trans, const GemvArgs &a, hipStream_t s) {
  if (a.ngroups == 0) return hipSuccess;
  const dim3 grid((unsigned)std::min<int64_t>(a.ngroups, 4096)), block(kThreads);
  if (cplx) {
    if (trans) hipLaunchKernelGGL((k_gemv<true, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_gemv<true, false>), grid, block, 0, s, a);
  } else {
    if (trans) hipLaunchKernelGGL((k_gemv<false, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_gemv<false, false>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

size_t dot_scratch_doubles() { return 2 * kDotBlocks; }

hipError_t launch_dot(bool cplx, bool conj, int64_t n, const double *x, const double *y,
                      double *part, double *out, hipStream_t s) {
  const dim3 grid(kDotBlocks), block(kThreads);
  if (cplx) {
    if (conj) hipLaunchKernelGGL((k_dot_part<true, true>), grid, block, 0, s, n, x, y, part);
    else hipLaunchKernelGGL((k_dot_part<true, false>), grid, block, 0, s, n, x, y, part);
  } else {
    hipLaunchKernelGGL((k_dot_part<false, false>), grid, block, 0, s, n, x, y, part);
  }
  hipLaunchKernelGGL(k_dot_final, dim3(1), block, 0, s, kDotBlocks, part, out);
  return hipGetLastError();
}

hipError_t launch_axpby(bool cplx, int64_t n, double ar, double ai, const double *x, double br,
                        double bi, double *y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const dim3 grid((unsigned)std::min<int64_t>((n + kThreads - 1) / kThreads, 4096)), block(kThreads);
  if (cplx) hipLaunchKernelGGL(k_axpby<true>, grid, block, 0, s, n, ar, ai, x, br, bi, y);
  else hipLaunchKernelGGL(k_axpby<false>, grid, block, 0, s, n, ar, ai, x, br, bi, y);
  return hipGetLastError();
}

hipError_t launch_mass(bool cplx, int32_t nt, const double *geo, int64_t ldg, double cr, double ci,
                       const double *x, double *y, hipStream_t s) {
  if (nt == 0) return hipSuccess;
  const dim3 grid((nt + kThreads - 1) / kThreads), block(kThreads);
  if (cplx) hipLaunchKernelGGL(k_mass<true>, grid, block, 0, s, nt, geo, ldg, cr, ci, x, y);
  else hipLaunchKernelGGL(k_mass<false>, grid, block, 0, s, nt, geo, ldg, cr, ci, x, y);
  return hipGetLastError();
}

}  // namespace bem
