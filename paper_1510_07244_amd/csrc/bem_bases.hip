// Cluster-basis kernels of the Green cross approximation (Sec. 2.3-2.4) for
// gfx950: the Green quadrature matrices A_t (kernel evaluations against the
// quadrature points of the Green box) and the basis contraction
// V_t = (A_t)[:, tau] (A_t)[t~, tau]^{-1} on the FP64 matrix cores.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "bem_device.h"

namespace bem {
namespace {

using namespace dev;

// ------------------------------------------------------------ Green matrix
// Entry (row triangle tau_i, Green point z_nu with normal n_nu, weight w_nu)
// of the two columns nu and m + nu (Sec. 2.3, eq. green_matrix):
//   side 0:  sqrt(w) int g(x, z) dx,        sqrt(w) delta int d/dn(z) g(x, z) dx
//   side 1:  sqrt(w) int d/dn(x) g(x, z) dx, sqrt(w) delta int d/dn(x) d/dn(z) g(x, z) dx
// (side 1 is the column basis of the double layer).  Triangle integrals use
// the Duffy rule: int_tau f = sqrt(g) sum_k w_k f(Phi(s_k, t_k)).
// A thread takes one row triangle and kGreenPerThread Green points: the rule
// points x_k on the triangle are formed once and used for every Green point.
constexpr int kGreenPerThread = 4;

template <int KERNEL, int SIDE>
__global__ __launch_bounds__(kThreads) void k_green(const GreenArgs a) {
  constexpr int J = kGreenPerThread;
  const int c = blockIdx.x;
  const int64_t rp0 = a.row_ptr[c], rp1 = a.row_ptr[c + 1];
  const int64_t off = a.out_off[c];
  const int64_t n = rp1 - rp0;
  const int m = a.m, mg = (m + J - 1) / J;
  const bool ok = rp0 >= 0 && rp0 <= rp1 && rp1 <= a.row_len && off >= 0 && off <= a.out_len &&
                  (n == 0 || 2 * (int64_t)m <= (a.out_len - off) / n);
  if (!ok) {
    if (threadIdx.x == 0) atomicOr(a.flags, FLAG_EINVAL);
    return;
  }
  const double delta = a.delta[c];
  const int64_t L = a.ldg;
  // the work items (row, group of J Green points) of one cluster are spread
  // over gridDim.y workgroups; consecutive threads take consecutive rows
  for (int64_t e = (int64_t)blockIdx.y * kThreads + threadIdx.x; e < n * mg;
       e += (int64_t)gridDim.y * kThreads) {
    const int64_t r = e % n;
    const int nu0 = (int)(e / n) * J;
    const int id = a.row_idx[rp0 + r];
    if (id < 0 || id >= a.nt) {
      atomicOr(a.flags, FLAG_EINVAL);
      continue;
    }
    double zx[J], zy[J], zz[J], mx[J], my[J], mz[J], wz[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int nu = min(nu0 + j, m - 1);  // past m: a copy, not written
      const double *zp = a.z + 3 * ((int64_t)c * m + nu);
      const double *np = a.zn + 3 * ((int64_t)c * m + nu);
      zx[j] = zp[0], zy[j] = zp[1], zz[j] = zp[2];
      mx[j] = np[0], my[j] = np[1], mz[j] = np[2];
      wz[j] = a.zw[(int64_t)c * m + nu];
    }
    const double v0x = a.geo[G_V0X * L + id], v0y = a.geo[G_V0Y * L + id], v0z = a.geo[G_V0Z * L + id];
    const double e1x = a.geo[G_E1X * L + id], e1y = a.geo[G_E1Y * L + id], e1z = a.geo[G_E1Z * L + id];
    const double e2x = a.geo[G_E2X * L + id], e2y = a.geo[G_E2Y * L + id], e2z = a.geo[G_E2Z * L + id];
    const double nx = a.geo[G_NX * L + id], ny = a.geo[G_NY * L + id], nz = a.geo[G_NZ * L + id];
    double pr[J], pi[J], qr[J], qi[J];  // + and - columns
#pragma unroll
    for (int j = 0; j < J; ++j) pr[j] = pi[j] = qr[j] = qi[j] = 0.0;
    for (int k = 0; k < a.nq; ++k) {
      const double s = a.rule[k], t = a.rule[a.nq + k], w = a.rule[2 * a.nq + k];
      // the rule point x = v0 + s e1 + t e2 on the triangle
      const double px = fma(s, e1x, fma(t, e2x, v0x));
      const double py = fma(s, e1y, fma(t, e2y, v0y));
      const double pz = fma(s, e1z, fma(t, e2z, v0z));
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const double dx = px - zx[j], dy = py - zy[j], dz = pz - zz[j];
        const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        const double iz = rsqrt_newton(r2);  // 1 / r
        const double i3 = iz * iz * iz;
        const double dnz = fma(dx, mx[j], fma(dy, my[j], dz * mz[j]));  // <x - z, n_z>
        const double dnx = fma(dx, nx, fma(dy, ny, dz * nz));           // <x - z, n_x>
        if constexpr (KERNEL == BEM_LAPLACE) {
          if constexpr (SIDE == 0) {
            pr[j] = fma(w, iz, pr[j]);
            qr[j] = fma(w, dnz * i3, qr[j]);
          } else {
            const double nn = fma(nx, mx[j], fma(ny, my[j], nz * mz[j]));
            pr[j] = fma(w, -dnx * i3, pr[j]);
            qr[j] = fma(w, fma(-3.0 * dnx * dnz, iz * iz, nn) * i3, qr[j]);
          }
        } else {
          const double r = r2 * iz, kr = a.kappa * r;
          double sn, cs;
          sincos_cw(kr, &sn, &cs);
          // e^{ikr} (1 - i kr) = (cs + kr sn) + i (sn - kr cs)
          const double ar = fma(kr, sn, cs), ai = fma(-kr, cs, sn);
          if constexpr (SIDE == 0) {
            pr[j] = fma(w * iz, cs, pr[j]);
            pi[j] = fma(w * iz, sn, pi[j]);
            qr[j] = fma(w * dnz * i3, ar, qr[j]);
            qi[j] = fma(w * dnz * i3, ai, qi[j]);
          } else {
            const double nn = fma(nx, mx[j], fma(ny, my[j], nz * mz[j]));
            pr[j] = fma(-w * dnx * i3, ar, pr[j]);
            pi[j] = fma(-w * dnx * i3, ai, pi[j]);
            // e^{ikr} [ (1 - i kr) nn / r^3 + (k^2 r^2 - 3 + 3 i kr) dnx dnz / r^5 ]
            const double u = dnx * dnz * iz * iz;
            const double br = fma(kr, kr, -3.0), bi = 3.0 * kr;
            const double tr = fma(nn, 1.0, u * br), ti = fma(-nn, kr, u * bi);  // (1 - i kr) nn + u (br + i bi)
            qr[j] = fma(w * i3, cs * tr - sn * ti, qr[j]);
            qi[j] = fma(w * i3, sn * tr + cs * ti, qi[j]);
          }
        }
      }
    }
    const double sg = a.geo[G_SG * L + id];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int nu = nu0 + j;
      if (nu >= m) break;
      const double sp = sqrt(wz[j]) * sg * kInv4Pi, sm = sp * delta;
      const int64_t ip = off + r + n * nu, im = off + r + n * (m + nu);
      if constexpr (KERNEL == BEM_LAPLACE) {
        static_cast<double *>(a.out)[ip] = pr[j] * sp;
        static_cast<double *>(a.out)[im] = qr[j] * sm;
      } else {
        static_cast<double2 *>(a.out)[ip] = make_double2(pr[j] * sp, pi[j] * sp);
        static_cast<double2 *>(a.out)[im] = make_double2(qr[j] * sm, qi[j] * sm);
      }
    }
  }
}

// ------------------------------------------------------- basis contraction
// V_c (n_c x k_c) = A_c[:, tau_c] (n_c x k_c) * P_c (k_c x k_c), all
// column-major, one workgroup per matrix, one wave per 16 x 16 output tile.
// v_mfma_f64_16x16x4_f64: lane l supplies A(l % 16, l / 16) and
// B(l / 16, l % 16) of a 16 x 4 by 4 x 16 product and holds
// D(l / 16 + 4 r, l % 16) in its four result registers r.
typedef double d4 __attribute__((ext_vector_type(4)));

template <bool CPLX>
__global__ __launch_bounds__(kThreads) void k_contract(const ContractArgs a) {
  const int c = blockIdx.x;
  const int n = a.nrows[c], k = a.rank[c], lda_cols = a.acols;
  const int64_t aoff = a.a_off[c], voff = a.v_off[c];
  if (n < 0 || k < 0 || k > a.max_rank || aoff < 0 || voff < 0 ||
      aoff + (int64_t)n * lda_cols > a.a_len || voff + (int64_t)n * k > a.v_len) {
    if (threadIdx.x == 0) atomicOr(a.flags, FLAG_EINVAL);
    return;
  }
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int32_t *tau = a.piv_cols + (int64_t)c * a.max_rank;
  const int64_t poff = (int64_t)c * a.max_rank * a.max_rank;
  const int ti = (n + 15) / 16, tj = (k + 15) / 16;
  const int li = lane & 15, lk = lane >> 4;
  constexpr int U = 4;  // k-steps whose operands are loaded before the MFMAs
  // the tiles of one matrix are spread over gridDim.y workgroups
  for (int tile = blockIdx.y * (kThreads / kWave) + wave; tile < ti * tj;
       tile += gridDim.y * (kThreads / kWave)) {
    const int i0 = (tile % ti) * 16, j0 = (tile / ti) * 16;
    const int row = i0 + li, col = j0 + li;
    d4 re = {0, 0, 0, 0}, im = {0, 0, 0, 0};
    for (int k0 = 0; k0 < k; k0 += 4 * U) {
      using T = typename std::conditional<CPLX, double2, double>::type;
      T av[U], bv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int kk = k0 + 4 * u + lk;
        int tc = kk < k ? tau[kk] : 0;
        if (tc < 0 || tc >= lda_cols) {  // never read outside A_c
          atomicOr(a.flags, FLAG_EINVAL);
          tc = 0;
        }
        const bool va = row < n && kk < k, vb = kk < k && col < k;
        const T *A = static_cast<const T *>(a.A);
        const T *P = reinterpret_cast<const T *>(a.pinv);
        av[u] = va ? A[aoff + row + (int64_t)n * tc] : T{};
        bv[u] = vb ? P[poff + kk + (int64_t)k * col] : T{};
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if constexpr (!CPLX) {
          re = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], re, 0, 0, 0);
        } else {
          re = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u].x, bv[u].x, re, 0, 0, 0);
          re = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[u].y, bv[u].y, re, 0, 0, 0);
          im = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u].x, bv[u].y, im, 0, 0, 0);
          im = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u].y, bv[u].x, im, 0, 0, 0);
        }
      }
    }
    for (int r = 0; r < 4; ++r) {
      const int row = i0 + lk + 4 * r, col = j0 + li;
      if (row < n && col < k) {
        if constexpr (!CPLX)
          static_cast<double *>(a.V)[voff + row + (int64_t)n * col] = re[r];
        else
          static_cast<double2 *>(a.V)[voff + row + (int64_t)n * col] = make_double2(re[r], im[r]);
      }
    }
  }
}

// ------------------------------------------------ pivot-block inverse
// P_c = A_c[t~_c, tau_c]^{-1} (k_c x k_c, column-major, leading dimension
// k_c) by in-place Gauss-Jordan elimination in the order of the cross
// approximation's pivots, one workgroup per matrix.  The matrix is
// X = M^T row-major (= M column-major), M[l][l'] = A_c[t~_c[l], tau_c[l']];
// row operations on X read and write contiguous rows, and the inverse of X
// left in place row-major is M^{-1} column-major.  The steps are sequential
// (k_c of them, two barriers each) and the data small: latency-bound, so the
// matrix stays in registers for the common ranks and the vector units serve
// it; the matrix cores are used by the contraction that follows.
template <bool CPLX>
struct Z;
template <>
struct Z<false> {
  double v;
  __device__ static Z make(double r, double) { Z z; z.v = r; return z; }
  __device__ double mag2() const { return v * v; }
  __device__ Z operator*(const Z &o) const { return make(v * o.v, 0); }
  __device__ Z operator-(const Z &o) const { return make(v - o.v, 0); }
  __device__ Z div(const Z &o) const { return make(v / o.v, 0); }
  __device__ bool finite_nonzero() const { return v != 0.0 && isfinite(v); }
  // the value of lane l (l uniform across the wave)
  __device__ Z lane_value(int l) const {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return make(__hiloint2double(hi, lo), 0);
  }
};
template <>
struct Z<true> {
  double re, im;
  __device__ static Z make(double r, double i) { Z z; z.re = r; z.im = i; return z; }
  __device__ double mag2() const { return re * re + im * im; }
  __device__ Z operator*(const Z &o) const { return make(re * o.re - im * o.im, re * o.im + im * o.re); }
  __device__ Z operator-(const Z &o) const { return make(re - o.re, im - o.im); }
  __device__ Z div(const Z &o) const {
    // (re + i im) / (a + i b) scaled by the larger of |a|, |b| (Smith)
    if (fabs(o.re) >= fabs(o.im)) {
      const double t = o.im / o.re, d = o.re + o.im * t;
      return make((re + im * t) / d, (im - re * t) / d);
    }
    const double t = o.re / o.im, d = o.re * t + o.im;
    return make((re * t + im) / d, (im * t - re) / d);
  }
  __device__ bool finite_nonzero() const {
    return (re != 0.0 || im != 0.0) && isfinite(re) && isfinite(im);
  }
  __device__ Z lane_value(int l) const {
    const int rl = __builtin_amdgcn_readlane(__double2loint(re), l);
    const int rh = __builtin_amdgcn_readlane(__double2hiint(re), l);
    const int il = __builtin_amdgcn_readlane(__double2loint(im), l);
    const int ih = __builtin_amdgcn_readlane(__double2hiint(im), l);
    return make(__hiloint2double(rh, rl), __hiloint2double(ih, il));
  }
};

constexpr int kInvMaxRank = 512;

// Gauss-Jordan on the k x k row-major matrix M (leading dimension ld, in
// global memory), in place and in the given order, without further
// pivoting: the pivots are the cross approximation's, each chosen as the
// largest entry of the residual of the whole Green matrix, so eliminating in
// their order is elimination with complete pivoting.  Two barriers per
// step: column s and the pivot row divided by the pivot are gathered into
// LDS, then every entry is updated by its own thread.
template <class T>
__device__ __forceinline__ void gauss_jordan(T *M, int ld, int k, T *fcol, T *ps,
                                             unsigned *flags) {
  const int tid = threadIdx.x, wave = tid / kWave, lane = tid & (kWave - 1);
  constexpr int W = kThreads / kWave;
  constexpr int kBatch = 8;  // rows per batch: the batch's loads issue together
  for (int s = 0; s < k; ++s) {
    const T piv = M[s * ld + s];
    if (tid == 0 && !piv.finite_nonzero()) atomicOr(flags, FLAG_NONFINITE);
    for (int r = tid; r < k; r += kThreads) {
      fcol[r] = M[r * ld + s];
      ps[r] = (r == s ? T::make(1, 0) : M[s * ld + r]).div(piv);
    }
    __syncthreads();
    for (int j = lane; j - lane < k; j += kWave) {  // uniform trip count
      const bool col = j < k;
      const T pj = col ? ps[j] : T::make(0, 0);
      for (int r0 = wave * kBatch; r0 < k; r0 += W * kBatch) {
        T fr[kBatch], old[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
          const int r = r0 + u;
          fr[u] = r < k && r != s ? fcol[r] : T::make(0, 0);
          old[u] = col && r < k && r != s && j != s ? M[r * ld + j] : T::make(0, 0);
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
          const int r = r0 + u;
          if (col && r < k) M[r * ld + j] = r == s ? pj : old[u] - fr[u] * pj;
        }
      }
    }
    __syncthreads();
  }
}

// One workgroup per matrix, in the matrix's global output slot: the ranks
// beyond the register-resident kernel's (real > 192, complex > 128), which
// an LDS copy could not hold either (160 KB).
template <bool CPLX>
__global__ __launch_bounds__(kThreads) void k_pivot_inverse(const PivInvArgs a, int reg_k) {
  using T = Z<CPLX>;
  __shared__ T fcol[kInvMaxRank], ps[kInvMaxRank];
  const int c = blockIdx.x;
  const int n = a.nrows[c], k = a.rank[c];
  if (k <= reg_k) return;  // uniform: done by the register-resident kernel
  const int64_t aoff = a.a_off[c];
  if (n < 0 || k < 0 || k > a.max_rank || k > n || aoff < 0 ||
      aoff + (int64_t)n * a.acols > a.a_len) {
    if (threadIdx.x == 0) atomicOr(a.flags, FLAG_EINVAL);
    return;
  }
  const int tid = threadIdx.x, wave = tid / kWave, lane = tid & (kWave - 1);
  constexpr int W = kThreads / kWave;
  const int32_t *prow = a.piv_rows + (int64_t)c * a.max_rank;
  const int32_t *pcol = a.piv_cols + (int64_t)c * a.max_rank;
  const T *A = reinterpret_cast<const T *>(a.A);
  T *X = reinterpret_cast<T *>(a.pinv) + (int64_t)c * a.max_rank * a.max_rank;
  // X[i][j] = M[j][i] = A[prow[j], pcol[i]]
  for (int i = wave; i < k; i += W) {
    const int ci = pcol[i];
    for (int j = lane; j < k; j += kWave) {
      const int rj = prow[j];
      T v = T::make(0, 0);
      if (ci < 0 || ci >= a.acols || rj < 0 || rj >= n) atomicOr(a.flags, FLAG_EINVAL);
      else v = A[aoff + rj + (int64_t)n * ci];
      X[(int64_t)i * k + j] = v;
    }
  }
  __syncthreads();
  gauss_jordan(X, k, k, fcol, ps, a.flags);
}

// Register-resident form for the common ranks: 16 waves (1024 threads); wave
// w holds rows w, w + 16, ... (RPW of them) and lane l columns l, l + 64, ...
// (CPL), so a matrix of up to 16 RPW = 64 CPL rows lives in registers for the
// whole elimination and LDS only carries, per step, column s and the pivot
// row.  Same steps and arithmetic as gauss_jordan; matrices of other sizes
// are left to k_pivot_inverse (the launcher runs both, each skipping the
// other's).
constexpr int kRegThreads = 1024;
constexpr int kRegWaves = kRegThreads / kWave;

template <bool CPLX, int RPW, int CPL>
__global__ __launch_bounds__(kRegThreads) void k_pivot_inverse_reg(const PivInvArgs a) {
  using T = Z<CPLX>;
  constexpr int KMAX = kRegWaves * RPW;
  static_assert(KMAX == kWave * CPL, "square register tile");
  __shared__ T fcol[KMAX], ps[KMAX];
  const int c = blockIdx.x;
  const int n = a.nrows[c], k = a.rank[c];
  if (k > KMAX) return;  // uniform: the LDS / global kernel takes it
  const int64_t aoff = a.a_off[c];
  if (n < 0 || k < 0 || k > a.max_rank || k > n || aoff < 0 ||
      aoff + (int64_t)n * a.acols > a.a_len) {
    if (threadIdx.x == 0) atomicOr(a.flags, FLAG_EINVAL);
    return;
  }
  const int tid = threadIdx.x, wave = tid / kWave, lane = tid & (kWave - 1);
  const int32_t *prow = a.piv_rows + (int64_t)c * a.max_rank;
  const int32_t *pcol = a.piv_cols + (int64_t)c * a.max_rank;
  const T *A = reinterpret_cast<const T *>(a.A);
  T *X = reinterpret_cast<T *>(a.pinv) + (int64_t)c * a.max_rank * a.max_rank;
  // X[r][j] = M[j][r] = A[prow[j], pcol[r]], r = wave + 16 i, j = lane + 64 q
  T x[RPW][CPL];
  int rj[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    const int j = lane + kWave * q;
    rj[q] = j < k ? prow[j] : 0;
    if (j < k && (rj[q] < 0 || rj[q] >= n)) atomicOr(a.flags, FLAG_EINVAL), rj[q] = 0;
  }
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const int r = wave + kRegWaves * i;
    int ci = r < k ? pcol[r] : 0;
    if (r < k && (ci < 0 || ci >= a.acols)) {
      if (lane == 0) atomicOr(a.flags, FLAG_EINVAL);
      ci = 0;
    }
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int j = lane + kWave * q;
      x[i][q] = r < k && j < k ? A[aoff + rj[q] + (int64_t)n * ci] : T::make(0, 0);
    }
  }
  for (int s = 0; s < k; ++s) {
    const int si = s / kRegWaves, sw = s % kRegWaves, sq = s / kWave, sl = s % kWave;
    // the pivot, from the lane that holds it, to the whole pivot row's wave
    T piv = T::make(0, 0);
    if (wave == sw) {
      T mine = T::make(0, 0);
#pragma unroll
      for (int i = 0; i < RPW; ++i)
#pragma unroll
        for (int q = 0; q < CPL; ++q)
          if (i == si && q == sq) mine = x[i][q];
      piv = mine.lane_value(sl);
      if (lane == 0 && !piv.finite_nonzero()) atomicOr(a.flags, FLAG_NONFINITE);
      // the pivot row divided by the pivot (its own entry: 1 / pivot)
#pragma unroll
      for (int q = 0; q < CPL; ++q) {
        const int j = lane + kWave * q;
        T v = T::make(0, 0);
#pragma unroll
        for (int i = 0; i < RPW; ++i)
          if (i == si) v = x[i][q];
        if (j < k) ps[j] = (j == s ? T::make(1, 0) : v).div(piv);
      }
    }
    // column s of every row, from the lanes that hold it
    if (lane == sl) {
#pragma unroll
      for (int i = 0; i < RPW; ++i) {
        const int r = wave + kRegWaves * i;
        T v = T::make(0, 0);
#pragma unroll
        for (int q = 0; q < CPL; ++q)
          if (q == sq) v = x[i][q];
        if (r < k) fcol[r] = v;
      }
    }
    __syncthreads();
    T pj[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int j = lane + kWave * q;
      pj[q] = j < k ? ps[j] : T::make(0, 0);
    }
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int r = wave + kRegWaves * i;
      const T fr = r < k ? fcol[r] : T::make(0, 0);
#pragma unroll
      for (int q = 0; q < CPL; ++q) {
        const int j = lane + kWave * q;
        if (r == s) x[i][q] = pj[q];
        else x[i][q] = (j == s ? T::make(0, 0) : x[i][q]) - fr * pj[q];
      }
    }
    __syncthreads();  // fcol and ps are rewritten by the next step
  }
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const int r = wave + kRegWaves * i;
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int j = lane + kWave * q;
      if (r < k && j < k) X[(int64_t)r * k + j] = x[i][q];
    }
  }
}

}  // namespace

hipError_t launch_pivot_inverse(bool cplx, const PivInvArgs &a, hipStream_t s) {
  if (a.nmat == 0) return hipSuccess;
  if (a.max_rank > kInvMaxRank) return hipErrorInvalidValue;
  const dim3 grid(a.nmat), block(kThreads);
  // ranks up to reg_k in registers (real 192 = 16 x 12 rows by 64 x 3
  // columns, complex 128 = 16 x 8 by 64 x 2), the rest in global memory
  const int reg_k = cplx ? kRegWaves * 8 : kRegWaves * 12;
  const dim3 rblock(kRegThreads);
  if (cplx) hipLaunchKernelGGL((k_pivot_inverse_reg<true, 8, 2>), grid, rblock, 0, s, a);
  else hipLaunchKernelGGL((k_pivot_inverse_reg<false, 12, 3>), grid, rblock, 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.max_rank <= reg_k) return e;
  if (cplx) hipLaunchKernelGGL((k_pivot_inverse<true>), grid, block, 0, s, a, reg_k);
  else hipLaunchKernelGGL((k_pivot_inverse<false>), grid, block, 0, s, a, reg_k);
  return hipGetLastError();
}

hipError_t launch_green(int kernel, int side, const GreenArgs &a, int grid_y, hipStream_t s) {
  if (a.ncl == 0) return hipSuccess;
  const dim3 grid(a.ncl, grid_y < 1 ? 1 : grid_y), block(kThreads);
  if (kernel == BEM_LAPLACE) {
    if (side == 0) hipLaunchKernelGGL((k_green<BEM_LAPLACE, 0>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_green<BEM_LAPLACE, 1>), grid, block, 0, s, a);
  } else {
    if (side == 0) hipLaunchKernelGGL((k_green<BEM_HELMHOLTZ, 0>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_green<BEM_HELMHOLTZ, 1>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_contract(bool cplx, const ContractArgs &a, int grid_y, hipStream_t s) {
  if (a.nmat == 0) return hipSuccess;
  const dim3 grid(a.nmat, grid_y < 1 ? 1 : grid_y), block(kThreads);
  if (cplx) hipLaunchKernelGGL((k_contract<true>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((k_contract<false>), grid, block, 0, s, a);
  return hipGetLastError();
}

}  // namespace bem
