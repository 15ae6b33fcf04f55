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
// (one 512-byte line per wave and column), and the waves of a workgroup work
// on different blocks without barriers between them.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "bem_device.h"

namespace bem {
namespace {

using namespace dev;

constexpr int kMaxVec = 512;  // longest output and input of one group / block

// v of lane k, k uniform across the wave (two scalar reads of the halves)
__device__ __forceinline__ double read_lane(double v, int k) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), k);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
  return __hiloint2double(hi, lo);
}

template <bool CPLX>
struct Num;
template <>
struct Num<false> {
  double v;
  __device__ static Num zero() { Num r; r.v = 0.0; return r; }
  __device__ void fma(const Num &m, const Num &x) { v = ::fma(m.v, x.v, v); }
  __device__ static Num load(const double *p, int64_t k) { Num r; r.v = p[k]; return r; }
  __device__ void add_to(double *p, int64_t k) const { p[k] += v; }
  __device__ void add(const Num &o) { v += o.v; }
  __device__ Num shfl_down_sum() const {
    Num r = *this;
    for (int o = kWave / 2; o >= 1; o >>= 1) r.v += __shfl_xor(r.v, o, kWave);
    return r;
  }
  // the value of lane k (k uniform across the wave)
  __device__ Num lane(int k) const { Num r; r.v = read_lane(v, k); return r; }
};
template <>
struct Num<true> {
  double re, im;
  __device__ static Num zero() { Num r; r.re = r.im = 0.0; return r; }
  __device__ void fma(const Num &m, const Num &x) {
    re = ::fma(m.re, x.re, re);
    re = ::fma(-m.im, x.im, re);
    im = ::fma(m.re, x.im, im);
    im = ::fma(m.im, x.re, im);
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
  __device__ Num lane(int k) const {
    Num r;
    r.re = read_lane(re, k);
    r.im = read_lane(im, k);
    return r;
  }
};

// Group g: y[out_idx[out_ptr[g] ..]] += sum_{b in group g} op(A_b) x[in_idx[in_ptr[b] ..]],
// op(A) = A (TRANS false; A is m_out x n_in) or A^T (TRANS true; A is
// n_in x m_out), column-major with the row count as leading dimension.  One
// workgroup of eight waves per group.  The group's work is cut into panels
// -- kPanel input columns of a block (TRANS false) or kPanel output columns
// (TRANS true), 16 real or 8 complex -- dealt to the waves in turn, so that a
// group of one small block still keeps every wave busy; a wave issues the
// loads of a panel before it uses them, since a product reads every matrix
// entry once and waits on memory.  TRANS false: lane l takes output rows
// l + 64 c of R consecutive chunks c in one pass (R = 2 when the group has
// more than 64 outputs: a coupling block of rank 65 .. 128 is one pass of
// 2 kPanel loads in flight per wave, not two passes of which the second
// runs with a few lanes); the panel's inputs are gathered one per lane and
// broadcast.  TRANS true: lane l takes input row l + 64 c, runs along the
// panel's columns and the wave adds each column's products up.  The waves'
// partial sums are added in wave order at the end: every sum runs in a
// fixed order, so results are reproducible bit for bit.
constexpr int kGemvThreads = 512;  // eight waves per group: more loads in flight

// TRANS false: this wave's panels of the group's blocks for the output rows
// of chunks c0 .. c0 + R - 1, into pw (the wave's row of partial sums).
template <bool CPLX, int R>
__device__ __forceinline__ void gemv_rows(const GemvArgs &a, int64_t m, int64_t b0, int64_t b1,
                                          int c0, int wave, int lane, Num<CPLX> *pw) {
  using T = Num<CPLX>;
  constexpr int kPanel = CPLX ? 8 : 16;
  constexpr int W = kGemvThreads / kWave;
  const double *A = static_cast<const double *>(a.A);
  const double *x = static_cast<const double *>(a.x);
  T acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = T::zero();
  int64_t task = 0;  // panels of the group's blocks so far
  for (int64_t b = b0; b < b1; ++b) {
    const int64_t i0 = a.in_ptr[b], i1 = a.in_ptr[b + 1], off = a.a_off[b];
    const int64_t n = i1 - i0;
    const int64_t np = (n + kPanel - 1) / kPanel;
    int64_t p = ((wave - task) % W + W) % W;  // this wave's first panel of block b
    task += np;
    if (p >= np) continue;
    if (!(i0 >= 0 && i0 <= i1 && i1 <= a.in_len && n <= kMaxVec && off >= 0 && off <= a.a_len &&
          (m == 0 || n <= (a.a_len - off) / m))) {
      if (lane == 0 && c0 == 0) atomicOr(a.flags, FLAG_EINVAL);
      continue;  // uniform in the wave
    }
    // the panel's inputs, one per lane (gathered one panel ahead, so that
    // the gather overlaps the current panel's matrix loads)
    auto gather = [&](int64_t q) {
      T v = T::zero();
      const int64_t j = q * kPanel + lane;
      if (lane < kPanel && j < n) {
        const int id = a.in_idx[i0 + j];
        if (id >= 0 && id < a.x_len) v = T::load(x, id);
        else if (c0 == 0) atomicOr(a.flags, FLAG_EINVAL);
      }
      return v;
    };
    T xl = gather(p);
    for (; p < np; p += W) {
      const int64_t j0 = p * kPanel;
      const int jn = (int)min((int64_t)kPanel, n - j0);
      // the panel's first column at a uniform address, the rest by 32-bit
      // offsets (m, n <= 512)
      const double *P = A + (CPLX ? 2 : 1) * (off + m * j0);
      const int mi = (int)m;
      T av[R][kPanel];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = lane + kWave * (c0 + r);
        const bool in = i < mi;
#pragma unroll
        for (int u = 0; u < kPanel; ++u)
          av[r][u] = in && u < jn ? T::load(P, i + mi * u) : T::zero();
      }
      const T xn = p + W < np ? gather(p + W) : T::zero();
#pragma unroll
      for (int u = 0; u < kPanel; ++u) {
        const T xu = xl.lane(u);
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r].fma(av[r][u], xu);
      }
      xl = xn;
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = lane + kWave * (int64_t)(c0 + r);
    if (i < m) pw[i] = acc[r];
  }
}

template <bool CPLX, bool TRANS>
__global__ __launch_bounds__(kGemvThreads, 1) void k_gemv(const GemvArgs a) {
  using T = Num<CPLX>;
  constexpr int kPanel = CPLX ? 8 : 16;
  __shared__ T part[kGemvThreads / kWave][kMaxVec];
  __shared__ T xw[TRANS ? kGemvThreads / kWave : 1][TRANS ? kMaxVec : 1];  // gathered inputs
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  constexpr int W = kGemvThreads / kWave;
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
    for (int64_t i = lane; i < m; i += kWave) part[wave][i] = T::zero();
    if (!TRANS) {
      // passes of two chunks of 64 output rows (one chunk if that is all)
      const int nchunks = (int)((m + kWave - 1) / kWave);
      if (nchunks <= 1) {
        gemv_rows<CPLX, 1>(a, m, b0, b1, 0, wave, lane, part[wave]);
      } else {
        for (int c0 = 0; c0 < nchunks; c0 += 2)
          gemv_rows<CPLX, 2>(a, m, b0, b1, c0, wave, lane, part[wave]);
      }
    } else {
      int64_t task = 0;  // panels of the group's blocks so far
      for (int64_t b = b0; b < b1; ++b) {
        const int64_t i0 = a.in_ptr[b], i1 = a.in_ptr[b + 1], off = a.a_off[b];
        const int64_t n = i1 - i0;
        const int64_t np = (m + kPanel - 1) / kPanel;
        int64_t p = ((wave - task) % W + W) % W;  // this wave's first panel of block b
        task += np;
        if (p >= np) continue;
        if (!(i0 >= 0 && i0 <= i1 && i1 <= a.in_len && n <= kMaxVec && off >= 0 &&
              off <= a.a_len && (m == 0 || n <= (a.a_len - off) / m))) {
          if (lane == 0) atomicOr(a.flags, FLAG_EINVAL);
          continue;  // uniform in the wave
        }
        // the block's inputs, gathered once for all of this wave's panels
        // into the wave's row of xw (each lane reads back only the rows it
        // wrote: no barrier)
        const int ni = (int)n;
        for (int i = lane; i < ni; i += kWave) {
          T v = T::zero();
          const int id = a.in_idx[i0 + i];
          if (id >= 0 && id < a.x_len) v = T::load(x, id);
          else atomicOr(a.flags, FLAG_EINVAL);
          xw[wave][i] = v;
        }
        for (; p < np; p += W) {
          const int64_t j0 = p * kPanel;
          const int jn = (int)min((int64_t)kPanel, m - j0);
          T s[kPanel];
#pragma unroll
          for (int u = 0; u < kPanel; ++u) s[u] = T::zero();
          const double *P = A + (CPLX ? 2 : 1) * (off + n * j0);
#pragma unroll 1
          for (int i = lane; i - lane < ni; i += kWave) {  // uniform trip count
            const T xi = i < ni ? xw[wave][i] : T::zero();
            T av[kPanel];
#pragma unroll
            for (int u = 0; u < kPanel; ++u)
              av[u] = i < ni && u < jn ? T::load(P, i + ni * u) : T::zero();
#pragma unroll
            for (int u = 0; u < kPanel; ++u) s[u].fma(av[u], xi);
          }
          // butterfly sums leave every column's total in every lane; lane
          // u adds output j0 + u
          T mine = T::zero();
#pragma unroll
          for (int u = 0; u < kPanel; ++u) {
            const T t = s[u].shfl_down_sum();
            if (lane == u) mine = t;
          }
          if (lane < jn) part[wave][j0 + lane].add(mine);
        }
      }
    }
    __syncthreads();
    for (int64_t k = tid; k < m; k += kGemvThreads) {
      T s = part[0][k];
      for (int w = 1; w < W; ++w) s.add(part[w][k]);
      const int id = a.out_idx[o0 + k];
      if (id < 0 || id >= a.y_len) atomicOr(a.flags, FLAG_EINVAL);
      else s.add_to(y, id);
    }
    __syncthreads();  // part is reused by the next group
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

// Conjugate-gradient updates with the step scalars in device memory (the
// layout of the state array is documented at bem_cg_step): the host reads
// them only to decide when to stop, not once per step.
__global__ __launch_bounds__(kThreads) void k_cg_xr(int64_t n, const double *st, const double *p,
                                                    const double *q, double *x, double *r) {
  const bool go = st[7] != 0.0 && st[2] != 0.0;
  const double alpha = go ? st[0] / st[2] : 0.0;
  const double one = 1.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    x[i] = alpha * p[i] + one * x[i];
    r[i] = -alpha * q[i] + one * r[i];
  }
}

__global__ __launch_bounds__(kThreads) void k_cg_p(int64_t n, const double *st, const double *r,
                                                   double *p) {
  if (!(st[7] != 0.0 && st[2] != 0.0)) return;  // uniform: stopped, p stays
  const double beta = st[4] / st[0];
  const double one = 1.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    p[i] = one * r[i] + beta * p[i];
}

__global__ void k_cg_close(double *st) {
  if (st[7] == 0.0) return;
  if (st[2] == 0.0) {  // p.q = 0: breakdown, stop with the current iterate
    st[7] = 0.0;
    return;
  }
  st[0] = st[4];
  st[8] += 1.0;
  st[7] = st[0] > st[6] && st[8] < st[9] ? 1.0 : 0.0;
}

}  // namespace

hipError_t launch_cg_step(int64_t n, double *state, double *x, double *r, double *p,
                          const double *q, double *dot_part, hipStream_t s) {
  const dim3 grid((unsigned)std::min<int64_t>(std::max<int64_t>((n + kThreads - 1) / kThreads, 1), 4096)),
      block(kThreads);
  hipLaunchKernelGGL(k_cg_xr, grid, block, 0, s, n, state, p, q, x, r);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_dot(false, false, n, r, r, dot_part, state + 4, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cg_p, grid, block, 0, s, n, state, r, p);
  hipLaunchKernelGGL(k_cg_close, dim3(1), dim3(1), 0, s, state);
  return hipGetLastError();
}

hipError_t launch_gemv(bool cplx, bool trans, const GemvArgs &a, hipStream_t s) {
  if (a.ngroups == 0) return hipSuccess;
  const dim3 grid((unsigned)std::min<int64_t>(a.ngroups, 4096)), block(kGemvThreads);
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
