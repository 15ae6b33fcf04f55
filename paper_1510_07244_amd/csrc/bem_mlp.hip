// Learned order selector (the learned form added to the method): a ReLU
// network 8 -> 64 -> 64 -> 64 -> n_out predicting, per regular pair, the
// log10 error of the Duffy/Gauss rule of Sec. 2.2 at orders 1 .. 6 against
// order 8.  Training in FP32 on the vector units (forward, reverse-mode
// gradient, Adam); inference in FP16 on the matrix cores
// (v_mfma_f32_16x16x16_f16, FP32 accumulation).
//
// Parameter vector (FP32): [mu(8), sigma(8), W1(64x8), b1, W2(64x64), b2,
// W3(64x64), b3, W4(n_out x 64), b4], W row-major; inputs are standardised
// as z = (x - mu) / sigma before the first layer.
#include <hip/hip_runtime.h>

#include "bem_device.h"

namespace bem {
namespace {

using namespace dev;

constexpr int kIn = 8, kHid = 64, kOutMax = 16;
constexpr int kSamples = 16;  // samples per workgroup of the gradient kernel

struct Off {
  int mu, sigma, w1, b1, w2, b2, w3, b3, w4, b4, total;
};
__host__ __device__ constexpr Off offsets(int n_out) {
  return Off{0,    8,    16,   528,  592,  4688, 4752, 8848, 8912, 8912 + 64 * n_out,
             8912 + 65 * n_out};
}

// ------------------------------------------------------------ training (FP32)
// h_out[s][o] = relu(b[o] + sum_k W[o][k] h_in[s][k]) for kSamples samples.
__device__ __forceinline__ void dense_relu(const float *W, const float *b, const float *in,
                                           int nin, float *out) {
  for (int e = threadIdx.x; e < kSamples * kHid; e += kThreads) {
    const int s = e / kHid, o = e % kHid;
    float a = b[o];
    for (int k = 0; k < nin; ++k) a = fmaf(W[o * nin + k], in[s * nin + k], a);
    out[e] = fmaxf(a, 0.0f);
  }
}

// Weight and bias gradients of one dense layer: gW[o][k] = sum_s d[s][o] in[s][k],
// gb[o] = sum_s d[s][o] (d: [kSamples][nout], in: [kSamples][nin]).
__device__ __forceinline__ void dense_grad(const float *d, int nout, const float *in, int nin,
                                           float *gW, float *gb) {
  for (int e = threadIdx.x; e < nout * nin; e += kThreads) {
    const int o = e / nin, k = e % nin;
    float a = 0.0f;
    for (int s = 0; s < kSamples; ++s) a = fmaf(d[s * nout + o], in[s * nin + k], a);
    gW[e] = a;
  }
  for (int o = threadIdx.x; o < nout; o += kThreads) {
    float a = 0.0f;
    for (int s = 0; s < kSamples; ++s) a += d[s * nout + o];
    gb[o] = a;
  }
}

// Back through a dense layer and the ReLU of its input:
// dprev[s][k] = (sum_o d[s][o] W[o][k]) * (h[s][k] > 0).
__device__ __forceinline__ void dense_back(const float *d, int nout, const float *W,
                                           const float *h, float *dprev) {
  for (int e = threadIdx.x; e < kSamples * kHid; e += kThreads) {
    const int s = e / kHid, k = e % kHid;
    float a = 0.0f;
    for (int o = 0; o < nout; ++o) a = fmaf(d[s * nout + o], W[o * kHid + k], a);
    dprev[e] = h[e] > 0.0f ? a : 0.0f;
  }
}

// One workgroup: forward and backward of kSamples samples; writes the sum of
// their gradient contributions (already divided by n * n_out) and of their
// squared errors.
__global__ __launch_bounds__(kThreads) void k_mlp_grad(int n_out, const float *__restrict__ P,
                                                       int64_t n, const float *__restrict__ x,
                                                       const float *__restrict__ t, float inv_count,
                                                       float *__restrict__ part,
                                                       float *__restrict__ lpart) {
  extern __shared__ float sm[];
  __shared__ float red[kThreads];
  const Off of = offsets(n_out);
  const int tot4 = (of.total + 3) & ~3;
  float *W = sm;
  float *z = W + tot4;                 // [kSamples][8]
  float *h1 = z + kSamples * kIn;      // [kSamples][64] each
  float *h2 = h1 + kSamples * kHid;
  float *h3 = h2 + kSamples * kHid;
  float *dy = h3 + kSamples * kHid;    // [kSamples][n_out]
  float *dA = dy + kSamples * kOutMax;
  float *dB = dA + kSamples * kHid;
  const int tid = threadIdx.x;
  const int64_t s0 = (int64_t)blockIdx.x * kSamples;
  for (int k = tid; k < of.total; k += kThreads) W[k] = P[k];
  __syncthreads();
  for (int e = tid; e < kSamples * kIn; e += kThreads) {
    const int s = e / kIn, f = e % kIn;
    z[e] = s0 + s < n ? (x[(s0 + s) * kIn + f] - W[of.mu + f]) / W[of.sigma + f] : 0.0f;
  }
  __syncthreads();
  dense_relu(W + of.w1, W + of.b1, z, kIn, h1);
  __syncthreads();
  dense_relu(W + of.w2, W + of.b2, h1, kHid, h2);
  __syncthreads();
  dense_relu(W + of.w3, W + of.b3, h2, kHid, h3);
  __syncthreads();
  float lsum = 0.0f;
  for (int e = tid; e < kSamples * n_out; e += kThreads) {
    const int s = e / n_out, o = e % n_out;
    float y = W[of.b4 + o];
    for (int k = 0; k < kHid; ++k) y = fmaf(W[of.w4 + o * kHid + k], h3[s * kHid + k], y);
    float d = 0.0f;
    if (s0 + s < n) {
      const float r = y - t[(s0 + s) * n_out + o];
      lsum = fmaf(r, r, lsum);
      d = 2.0f * r * inv_count;
    }
    dy[e] = d;
  }
  red[tid] = lsum;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) lpart[blockIdx.x] = red[0];
  float *G = part + (int64_t)blockIdx.x * of.total;
  for (int k = tid; k < 2 * kIn; k += kThreads) G[k] = 0.0f;  // mu, sigma: not trained
  dense_grad(dy, n_out, h3, kHid, G + of.w4, G + of.b4);
  dense_back(dy, n_out, W + of.w4, h3, dA);
  __syncthreads();
  dense_grad(dA, kHid, h2, kHid, G + of.w3, G + of.b3);
  dense_back(dA, kHid, W + of.w3, h2, dB);
  __syncthreads();
  dense_grad(dB, kHid, h1, kHid, G + of.w2, G + of.b2);
  dense_back(dB, kHid, W + of.w2, h1, dA);
  __syncthreads();
  dense_grad(dA, kHid, z, kIn, G + of.w1, G + of.b1);
}

// grad[p] = sum over workgroups (in order) of part[wg][p]; loss likewise.
__global__ void k_mlp_reduce(int total, int nwg, const float *__restrict__ part,
                             const float *__restrict__ lpart, float inv_count,
                             float *__restrict__ grad, float *__restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < total) {
    float a = 0.0f;
    for (int w = 0; w < nwg; ++w) a += part[(int64_t)w * total + p];
    grad[p] = a;
  }
  if (p == 0 && loss) {
    float a = 0.0f;
    for (int w = 0; w < nwg; ++w) a += lpart[w];
    *loss = a * inv_count;
  }
}

__global__ void k_mlp_adam(int64_t np, float *__restrict__ p, const float *__restrict__ g,
                           float *__restrict__ m, float *__restrict__ v, float lr, float b1,
                           float b2, float eps, float c1, float c2) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= np) return;
  const float gk = g[k];
  const float mk = fmaf(b1, m[k], (1.0f - b1) * gk);
  const float vk = fmaf(b2, v[k], (1.0f - b2) * gk * gk);
  m[k] = mk;
  v[k] = vk;
  p[k] -= lr * (mk * c1) / (sqrtf(vk * c2) + eps);
}

// FP32 forward, one sample per thread (weights read as uniform scalars).
__global__ __launch_bounds__(kThreads) void k_mlp_fwd32(int n_out, const float *__restrict__ P,
                                                        int64_t n, const float *__restrict__ x,
                                                        float *__restrict__ y) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const Off of = offsets(n_out);
  typedef const float __attribute__((address_space(4))) *cptr;
  const cptr W = (cptr)P;
  float z[kIn], h1[kHid], h2[kHid], out[kOutMax];
  for (int f = 0; f < kIn; ++f) z[f] = (x[s * kIn + f] - W[of.mu + f]) / W[of.sigma + f];
  for (int o = 0; o < kHid; ++o) {
    float a = W[of.b1 + o];
    for (int k = 0; k < kIn; ++k) a = fmaf(W[of.w1 + o * kIn + k], z[k], a);
    h1[o] = fmaxf(a, 0.0f);
  }
  for (int o = 0; o < kHid; ++o) {
    float a = W[of.b2 + o];
    for (int k = 0; k < kHid; ++k) a = fmaf(W[of.w2 + o * kHid + k], h1[k], a);
    h2[o] = fmaxf(a, 0.0f);
  }
  for (int o = 0; o < kOutMax; ++o) out[o] = o < n_out ? W[of.b4 + o] : 0.0f;
  for (int j = 0; j < kHid; ++j) {
    float a = W[of.b3 + j];
    for (int k = 0; k < kHid; ++k) a = fmaf(W[of.w3 + j * kHid + k], h2[k], a);
    a = fmaxf(a, 0.0f);
    for (int o = 0; o < kOutMax; ++o)
      if (o < n_out) out[o] = fmaf(W[of.w4 + o * kHid + j], a, out[o]);
  }
  for (int o = 0; o < n_out; ++o) y[s * n_out + o] = out[o];
}

// ------------------------------------------------------------ inference (FP16)
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Row of the 16 x 16 result held by lane group g (= lane / 16) in result
// register r of v_mfma_f32_16x16x16_f16; the column is lane % 16.
__device__ __forceinline__ constexpr int drow(int g, int r) { return 4 * g + r; }

// The network's weights as matrix-core operands of one wave.  Layers are
// computed transposed, H^T = W Z^T: the weights are the A operand (lane
// holds row lane % 16, k-slots of its lane group) and the activations of 16
// samples the B operand (lane holds sample lane % 16), so that a layer's
// result registers are directly the next layer's B operand when slot (g, j)
// of the A operand carries k index drow(g, j).
struct Net16 {
  h4 a1[4], a2[4][4], a3[4][4], a4[4];
  f4 c1[4], c2[4], c3[4], c4;  // biases in result layout
  float mu[4], isg[4];         // this lane's input standardisation (lane group 0, 1)
};

__device__ __forceinline__ void load_net(const float *__restrict__ P, int n_out, Net16 *N) {
  const Off of = offsets(n_out);
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
  for (int mt = 0; mt < 4; ++mt) {
    const int row = mt * 16 + c;
    for (int j = 0; j < 4; ++j) {
      const int f = 4 * g + j;  // input feature of slot (g, j)
      N->a1[mt][j] = (_Float16)(g < 2 ? P[of.w1 + row * kIn + f] : 0.0f);
    }
    for (int kt = 0; kt < 4; ++kt)
      for (int j = 0; j < 4; ++j) {
        const int k = kt * 16 + drow(g, j);
        N->a2[mt][kt][j] = (_Float16)P[of.w2 + row * kHid + k];
        N->a3[mt][kt][j] = (_Float16)P[of.w3 + row * kHid + k];
      }
    for (int r = 0; r < 4; ++r) {
      const int o = mt * 16 + drow(g, r);
      N->c1[mt][r] = P[of.b1 + o];
      N->c2[mt][r] = P[of.b2 + o];
      N->c3[mt][r] = P[of.b3 + o];
    }
  }
  for (int kt = 0; kt < 4; ++kt)
    for (int j = 0; j < 4; ++j)
      N->a4[kt][j] = (_Float16)(c < n_out ? P[of.w4 + c * kHid + kt * 16 + drow(g, j)] : 0.0f);
  for (int r = 0; r < 4; ++r) {
    const int o = drow(g, r);
    N->c4[r] = o < n_out ? P[of.b4 + o] : 0.0f;
  }
  for (int j = 0; j < 4; ++j) {
    const int f = (4 * g + j) & 7;
    N->mu[j] = P[of.mu + f];
    N->isg[j] = 1.0f / P[of.sigma + f];
  }
}

__device__ __forceinline__ h4 relu_h4(f4 v) {
  h4 r;
  for (int j = 0; j < 4; ++j) r[j] = (_Float16)fmaxf(v[j], 0.0f);
  return r;
}

// Network outputs for the 16 samples of a wave-group.  `feat` holds this
// lane's four raw inputs (features 4g .. 4g+3 of sample lane % 16; unused
// for lane groups 2, 3).  Returns the result registers: output drow(g, r)
// of sample lane % 16.
__device__ __forceinline__ f4 net16(const Net16 &N, const float feat[4]) {
  const int g = (threadIdx.x & 63) >> 4;
  h4 b;
  for (int j = 0; j < 4; ++j)
    b[j] = (_Float16)(g < 2 ? (feat[j] - N.mu[j]) * N.isg[j] : 0.0f);
  h4 hb1[4], hb2[4], hb3[4];
  for (int mt = 0; mt < 4; ++mt)
    hb1[mt] = relu_h4(__builtin_amdgcn_mfma_f32_16x16x16f16(N.a1[mt], b, N.c1[mt], 0, 0, 0));
  for (int mt = 0; mt < 4; ++mt) {
    f4 acc = N.c2[mt];
    for (int kt = 0; kt < 4; ++kt)
      acc = __builtin_amdgcn_mfma_f32_16x16x16f16(N.a2[mt][kt], hb1[kt], acc, 0, 0, 0);
    hb2[mt] = relu_h4(acc);
  }
  for (int mt = 0; mt < 4; ++mt) {
    f4 acc = N.c3[mt];
    for (int kt = 0; kt < 4; ++kt)
      acc = __builtin_amdgcn_mfma_f32_16x16x16f16(N.a3[mt][kt], hb2[kt], acc, 0, 0, 0);
    hb3[mt] = relu_h4(acc);
  }
  f4 acc = N.c4;
  for (int kt = 0; kt < 4; ++kt)
    acc = __builtin_amdgcn_mfma_f32_16x16x16f16(N.a4[kt], hb3[kt], acc, 0, 0, 0);
  return acc;
}

// Generic inference over stored inputs x[n][8] -> y[n][n_out].
__global__ __launch_bounds__(kThreads) void k_mlp_infer16(int n_out, const float *__restrict__ P,
                                                          int64_t n, const float *__restrict__ x,
                                                          float *__restrict__ y) {
  Net16 N;
  load_net(P, n_out, &N);
  const int l = threadIdx.x & 63, g = l >> 4;
  const int64_t nwaves = (int64_t)gridDim.x * (kThreads / kWave);
  const int64_t w0 = (int64_t)blockIdx.x * (kThreads / kWave) + threadIdx.x / kWave;
  for (int64_t s0 = w0 * 16; s0 < n; s0 += nwaves * 16) {
    const int64_t s = s0 + (l & 15);
    float f[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (g < 2 && s < n)
      for (int j = 0; j < 4; ++j) f[j] = x[s * kIn + 4 * g + j];
    const f4 out = net16(N, f);
    for (int r = 0; r < 4; ++r) {
      const int o = drow(g, r);
      if (s < n && o < n_out) y[s * n_out + o] = out[r];
    }
  }
}

// ------------------------------------------------------------ pair inputs
// Inputs of a regular pair (i, j) from the triangle geometry (FP64, then
// rounded to FP32): see the selector's definition in the header.
__device__ __forceinline__ void pair_features(const double *g, int64_t L, int i, int j,
                                              int layer, double kappa, float f[8]) {
  double ci[3], cj[3], ni[3], nj[3];
  double di = 0.0, dj = 0.0;
  {
    double a2 = 0, b2 = 0, s2 = 0, c2 = 0, d2 = 0, t2 = 0;
    for (int c = 0; c < 3; ++c) {
      const double e1i = g[(G_E1X + c) * L + i], e2i = g[(G_E2X + c) * L + i];
      const double e1j = g[(G_E1X + c) * L + j], e2j = g[(G_E2X + c) * L + j];
      ci[c] = g[(G_V0X + c) * L + i] + (2.0 * e1i + e2i) / 3.0;
      cj[c] = g[(G_V0X + c) * L + j] + (2.0 * e1j + e2j) / 3.0;
      ni[c] = g[(G_NX + c) * L + i];
      nj[c] = g[(G_NX + c) * L + j];
      a2 = fma(e1i, e1i, a2);
      b2 = fma(e2i, e2i, b2);
      s2 = fma(e1i + e2i, e1i + e2i, s2);
      c2 = fma(e1j, e1j, c2);
      d2 = fma(e2j, e2j, d2);
      t2 = fma(e1j + e2j, e1j + e2j, t2);
    }
    di = sqrt(fmax(a2, fmax(b2, s2)));
    dj = sqrt(fmax(c2, fmax(d2, t2)));
  }
  const double ai = 0.5 * g[G_SG * L + i], aj = 0.5 * g[G_SG * L + j];
  const double D = fmax(di, dj);
  const double s0 = ci[0] - cj[0], s1 = ci[1] - cj[1], s2 = ci[2] - cj[2];
  const double r = sqrt(fma(s0, s0, fma(s1, s1, s2 * s2)));
  const double q = 0.4330127018922193;  // sqrt(3) / 4
  f[0] = (float)log(r / D);
  f[1] = (float)(q * di * di / ai);
  f[2] = (float)(q * dj * dj / aj);
  f[3] = (float)(fmin(ai, aj) / fmax(ai, aj));
  f[4] = (float)(kappa * D);
  f[5] = (float)fma(ni[0], nj[0], fma(ni[1], nj[1], ni[2] * nj[2]));
  f[6] = (float)layer;
  f[7] = (float)fabs(fma(s0, nj[0], fma(s1, nj[1], s2 * nj[2])) / r);
}

template <int KERNEL, int LAYER>
__device__ __forceinline__ double entry_abs_diff(const Acc<KERNEL> &a, const Acc<KERNEL> &b) {
  if constexpr (KERNEL == BEM_LAPLACE) return fabs(a.re - b.re);
  else return hypot(a.re - b.re, a.im - b.im);
}

template <int KERNEL>
__device__ __forceinline__ double entry_abs(const Acc<KERNEL> &a) {
  if constexpr (KERNEL == BEM_LAPLACE) return fabs(a.re);
  else return hypot(a.re, a.im);
}

// Training samples: inputs and targets e_q, q = 1 .. 6, of regular pairs.
template <int KERNEL, int LAYER>
__global__ __launch_bounds__(kThreads) void k_selector_samples(const SampleArgs a) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.n) return;
  const int i = a.rows[k], j = a.cols[k];
  bool ok = i >= 0 && i < a.nt && j >= 0 && j < a.nt;
  if (ok) {
    const int *ti = a.tri + 3 * (int64_t)i, *tj = a.tri + 3 * (int64_t)j;
    ok = shared_vertex_count(ti[0], ti[1], ti[2], tj[0], tj[1], tj[2]) == 0;
  }
  if (!ok) {
    atomicOr(a.flags, FLAG_EINVAL);
    for (int f = 0; f < kIn; ++f) a.x[k * kIn + f] = __builtin_nanf("");
    for (int q = 0; q < kSelQ; ++q) a.t[k * kSelQ + q] = __builtin_nanf("");
    return;
  }
  float f[8];
  pair_features(a.geo, a.ldg, i, j, LAYER, a.kappa, f);
  for (int c = 0; c < kIn; ++c) a.x[k * kIn + c] = f[c];
  const Acc<KERNEL> ref = regular_pair_fp64<KERNEL, LAYER>(a.geo, a.ldg, a.rule[kSelQ], a.nq[kSelQ],
                                                          a.kappa, i, j);
  // size of a single-layer entry of the pair: |tau_i| |tau_j| / (4 pi r)
  double r2 = 0.0;
  for (int c = 0; c < 3; ++c) {
    const double d = (a.geo[(G_V0X + c) * a.ldg + i] +
                      (2.0 * a.geo[(G_E1X + c) * a.ldg + i] + a.geo[(G_E2X + c) * a.ldg + i]) / 3.0) -
                     (a.geo[(G_V0X + c) * a.ldg + j] +
                      (2.0 * a.geo[(G_E1X + c) * a.ldg + j] + a.geo[(G_E2X + c) * a.ldg + j]) / 3.0);
    r2 = fma(d, d, r2);
  }
  const double s = 0.25 * a.geo[G_SG * a.ldg + i] * a.geo[G_SG * a.ldg + j] * kInv4Pi / sqrt(r2);
  const double den = fmax(entry_abs<KERNEL>(ref), 1e-3 * s);
  for (int q = 0; q < kSelQ; ++q) {
    const Acc<KERNEL> v = regular_pair_fp64<KERNEL, LAYER>(a.geo, a.ldg, a.rule[q], a.nq[q],
                                                          a.kappa, i, j);
    a.t[k * kSelQ + q] = (float)log10(fmax(entry_abs_diff<KERNEL, LAYER>(v, ref) / den, 1e-16));
  }
}

// Lane group and result register holding output o (inverse of drow).
__device__ __forceinline__ constexpr int dgroup(int o) { return o / 4; }
__device__ __forceinline__ constexpr int dreg(int o) { return o % 4; }

// Orders of the entries of near-field blocks: 0 for pairs with a common
// vertex, else the smallest order in [q_min, q_plain - 1] whose predicted
// error plus the margin is at most log10(tol) at it and at every order above
// it below q_plain; q_plain when q_plain - 1 fails.  One workgroup per block;
// each wave takes 16 entries at a time.
__global__ __launch_bounds__(kThreads) void k_select_orders(const SelectArgs a) {
  const int b = blockIdx.x;
  const int64_t rp0 = a.row_ptr[b], rp1 = a.row_ptr[b + 1];
  const int64_t cp0 = a.col_ptr[b], cp1 = a.col_ptr[b + 1];
  const int64_t off = a.out_off[b];
  bool ok = rp0 >= 0 && rp0 <= rp1 && rp1 <= a.row_len && cp0 >= 0 && cp0 <= cp1 &&
            cp1 <= a.col_len && off >= 0 && off <= a.out_len;
  const int64_t nr = rp1 - rp0, nc = cp1 - cp0;
  ok = ok && (nr == 0 || nc <= (a.out_len - off) / nr);
  if (!ok) {
    if (threadIdx.x == 0) atomicOr(a.flags, FLAG_EINVAL);
    return;
  }
  Net16 N;
  load_net(a.params, kSelQ, &N);
  const int l = threadIdx.x & 63, g = l >> 4, wave = threadIdx.x / kWave;
  const int64_t ne = nr * nc;
  for (int64_t e0 = (int64_t)wave * 16; e0 < ne; e0 += 16 * (kThreads / kWave)) {
    const int64_t e = e0 + (l & 15);
    const bool live = e < ne;
    int i = -1, j = -1, cls = 1;
    if (live) {
      i = a.row_idx[rp0 + e % nr];
      j = a.col_idx[cp0 + e / nr];
      if (i < 0 || i >= a.nt || j < 0 || j >= a.nt) {
        atomicOr(a.flags, FLAG_EINVAL);
        i = -1;
      } else {
        const int *ti = a.tri + 3 * (int64_t)i, *tj = a.tri + 3 * (int64_t)j;
        cls = shared_vertex_count(ti[0], ti[1], ti[2], tj[0], tj[1], tj[2]);
      }
    }
    float f[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (i >= 0 && cls == 0 && g < 2) {
      float all[8];
      pair_features(a.geo, a.ldg, i, j, a.layer, a.kappa, all);
      for (int c = 0; c < 4; ++c) f[c] = all[4 * g + c];
    }
    const f4 out = net16(N, f);
    // gather the kSelQ outputs of sample l % 16 into lane group 0
    float pred[kSelQ];
    for (int o = 0; o < kSelQ; ++o) pred[o] = __shfl(out[dreg(o)], dgroup(o) * 16 + (l & 15), kWave);
    if (g == 0 && i >= 0) {
      int q = 0;
      if (cls == 0) {
        q = a.q_plain;
        bool run = true;
        for (int qq = a.q_plain - 1; qq >= a.q_min; --qq) {
          run = run && pred[qq - 1] + a.margin <= a.log_tol;
          if (run) q = qq;
        }
      }
      a.orders[off + e] = (int8_t)q;
    }
  }
}

}  // namespace

hipError_t launch_mlp_grad(int n_out, const float *P, int64_t n, const float *x, const float *t,
                           float *part, float *lpart, float *grad, float *loss, hipStream_t s) {
  const Off of = offsets(n_out);
  const int nwg = (int)((n + kSamples - 1) / kSamples);
  const float inv = (float)(1.0 / ((double)n * n_out));
  const size_t lds = sizeof(float) * (((of.total + 3) & ~3) + kSamples * kIn + 3 * kSamples * kHid +
                                      kSamples * kOutMax + 2 * kSamples * kHid);
  hipLaunchKernelGGL(k_mlp_grad, dim3(nwg), dim3(kThreads), lds, s, n_out, P, n, x, t, inv, part,
                     lpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_reduce, dim3((of.total + 255) / 256), dim3(256), 0, s, of.total, nwg,
                     part, lpart, inv, grad, loss);
  return hipGetLastError();
}

size_t mlp_grad_scratch_floats(int n_out, int64_t n) {
  const int64_t nwg = (n + kSamples - 1) / kSamples;
  return (size_t)nwg * (offsets(n_out).total + 1);
}

int mlp_params(int n_out) { return offsets(n_out).total; }

hipError_t launch_mlp_adam(int64_t np, float *p, const float *g, float *m, float *v, float lr,
                           float b1, float b2, float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_adam, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, np, p, g, m,
                     v, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(bool f16, int n_out, const float *P, int64_t n, const float *x,
                              float *y, hipStream_t s) {
  if (f16) {
    const int64_t groups = (n + 15) / 16;
    const unsigned grid = (unsigned)std::min<int64_t>((groups + 3) / 4, 2048);
    hipLaunchKernelGGL(k_mlp_infer16, dim3(grid), dim3(kThreads), 0, s, n_out, P, n, x, y);
  } else {
    hipLaunchKernelGGL(k_mlp_fwd32, dim3((unsigned)((n + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, n_out, P, n, x, y);
  }
  return hipGetLastError();
}

hipError_t launch_selector_samples(int kernel, int layer, const SampleArgs &a, hipStream_t s) {
  const dim3 grid((unsigned)((a.n + kThreads - 1) / kThreads)), block(kThreads);
  if (kernel == BEM_LAPLACE) {
    if (layer == BEM_SLP) hipLaunchKernelGGL((k_selector_samples<BEM_LAPLACE, BEM_SLP>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_selector_samples<BEM_LAPLACE, BEM_DLP>), grid, block, 0, s, a);
  } else {
    if (layer == BEM_SLP) hipLaunchKernelGGL((k_selector_samples<BEM_HELMHOLTZ, BEM_SLP>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_selector_samples<BEM_HELMHOLTZ, BEM_DLP>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_select_orders(const SelectArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_select_orders, dim3(a.nblocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace bem
