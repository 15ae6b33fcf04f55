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
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

// v_mfma_f32_16x16x32_f16 (read on the device with an in-bounds probe): the
// A operand of lane l holds row l % 16 at the eight k-slots (g, j) of its
// lane group g = l / 16, the B operand column l % 16 at the same slots, and
// result register r holds row 4 g + r, column l % 16.
__device__ __forceinline__ constexpr int drow(int g, int r) { return 4 * g + r; }

// Layers are computed transposed, H^T = W Z^T: the weights are the A operand
// and the activations of 16 samples the B operand.  For a 64-wide layer the
// B operand of k-step ks (32 neurons) is the result registers of tiles 2 ks
// and 2 ks + 1, so A's slot (g, j) carries neuron kidx(ks, g, j).
__device__ __forceinline__ constexpr int kidx(int ks, int g, int j) {
  return ks * 32 + (j < 4 ? drow(g, j) : 16 + drow(g, j - 4));
}

struct Net16 {
  h8 a1[4], a2[4][2], a3[4][2], a4[2];
};

// Biases in LDS: b1, b2, b3 (64 each), b4 (16, zero padded); input
// standardisation mu and 1 / sigma (8 each).
constexpr int kBiasFloats = 3 * kHid + kOutMax + 2 * kIn;

// A operands of the network for lane l of a wave.
__device__ __forceinline__ void build_net(const float *__restrict__ P, int n_out, int l, Net16 *N) {
  const Off of = offsets(n_out);
  const int g = l >> 4, c = l & 15;
  for (int mt = 0; mt < 4; ++mt) {
    const int row = mt * 16 + c;
    for (int j = 0; j < 8; ++j)
      N->a1[mt][j] = (_Float16)(g == 0 ? P[of.w1 + row * kIn + j] : 0.0f);
    for (int ks = 0; ks < 2; ++ks)
      for (int j = 0; j < 8; ++j) {
        N->a2[mt][ks][j] = (_Float16)P[of.w2 + row * kHid + kidx(ks, g, j)];
        N->a3[mt][ks][j] = (_Float16)P[of.w3 + row * kHid + kidx(ks, g, j)];
      }
  }
  for (int ks = 0; ks < 2; ++ks)
    for (int j = 0; j < 8; ++j)
      N->a4[ks][j] = (_Float16)(c < n_out ? P[of.w4 + c * kHid + kidx(ks, g, j)] : 0.0f);
}

// Packed network: kNetSlots FP16 operand vectors per lane, slot-major
// ([slot][64 lanes], 16 bytes each), then kBiasFloats floats (biases, mu,
// 1 / sigma).  Built once per call by one wave (k_pack_net) and read by every
// wave of the inference kernels with 16-byte loads.  Slots 0..21 are Net16;
// slots 22 + 2 G + ks hold the output layer with its rows rotated by 4 G
// (output o at row (o + 4 G) mod 16), so that group G of a four-group step
// leaves outputs 0..3 of its samples in lane group G.
constexpr int kNetSlots = 30;
constexpr int kRotSlot = 22;

__global__ void k_pack_net(int n_out, const float *__restrict__ P, h8 *__restrict__ packed) {
  const int l = threadIdx.x;
  Net16 N;
  build_net(P, n_out, l, &N);
  int k = 0;
  for (int mt = 0; mt < 4; ++mt) packed[(k++) * 64 + l] = N.a1[mt];
  for (int mt = 0; mt < 4; ++mt)
    for (int ks = 0; ks < 2; ++ks) packed[(k++) * 64 + l] = N.a2[mt][ks];
  for (int mt = 0; mt < 4; ++mt)
    for (int ks = 0; ks < 2; ++ks) packed[(k++) * 64 + l] = N.a3[mt][ks];
  for (int ks = 0; ks < 2; ++ks) packed[(k++) * 64 + l] = N.a4[ks];
  const Off of = offsets(n_out);
  const int g = l >> 4, c = l & 15;
  for (int G = 0; G < 4; ++G)
    for (int ks = 0; ks < 2; ++ks) {
      const int o = (c - 4 * G) & 15;
      h8 v;
      for (int j = 0; j < 8; ++j)
        v[j] = (_Float16)(o < n_out ? P[of.w4 + o * kHid + kidx(ks, g, j)] : 0.0f);
      packed[(k++) * 64 + l] = v;
    }
  float *bias = reinterpret_cast<float *>(packed + kNetSlots * 64);
  for (int q = l; q < kBiasFloats; q += 64) {
    float v;
    if (q < 3 * kHid) v = P[(q < kHid ? of.b1 : q < 2 * kHid ? of.b2 - kHid : of.b3 - 2 * kHid) + q];
    else if (q < 3 * kHid + kOutMax) v = q - 3 * kHid < n_out ? P[of.b4 + q - 3 * kHid] : 0.0f;
    else if (q < 3 * kHid + kOutMax + kIn) v = P[of.mu + q - 3 * kHid - kOutMax];
    else v = 1.0f / P[of.sigma + q - 3 * kHid - kOutMax - kIn];
    bias[q] = v;
  }
}

// This lane's operands from the packed network, the biases into LDS.
__device__ __forceinline__ void load_net(const h8 *__restrict__ packed, Net16 *N, float *bias) {
  const int l = threadIdx.x & 63;
  int k = 0;
  for (int mt = 0; mt < 4; ++mt) N->a1[mt] = packed[(k++) * 64 + l];
  for (int mt = 0; mt < 4; ++mt)
    for (int ks = 0; ks < 2; ++ks) N->a2[mt][ks] = packed[(k++) * 64 + l];
  for (int mt = 0; mt < 4; ++mt)
    for (int ks = 0; ks < 2; ++ks) N->a3[mt][ks] = packed[(k++) * 64 + l];
  for (int ks = 0; ks < 2; ++ks) N->a4[ks] = packed[(k++) * 64 + l];
  const float *gb = reinterpret_cast<const float *>(packed + kNetSlots * 64);
  for (int q = threadIdx.x; q < kBiasFloats; q += blockDim.x) bias[q] = gb[q];
}

__device__ __forceinline__ f4 bias4(const float *bias, int base, int g) {
  return *reinterpret_cast<const f4 *>(bias + base + drow(g, 0));
}

// ReLU after the FP16 rounding, on the bit patterns: a negative half (sign
// bit set, -0 included) is a negative int16, so a packed integer max with 0
// gives exactly the rounding of max(x, 0) for every finite x.
typedef short s2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef _Float16 hf2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t relu2(float a, float b) {
  const hf2 h = __builtin_convertvector((f2){a, b}, hf2);
  const s2 zero = {0, 0};
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s2, h), zero));
}
__device__ __forceinline__ h8 relu_pair(f4 lo, f4 hi) {
  const uint32_t w[4] = {relu2(lo[0], lo[1]), relu2(lo[2], lo[3]), relu2(hi[0], hi[1]),
                         relu2(hi[2], hi[3])};
  return __builtin_bit_cast(h8, w);
}

// Standardised FP16 inputs of one sample (the same arithmetic everywhere).
__device__ __forceinline__ h8 standardise(const float x[8], const float *bias) {
  const float *mu = bias + 3 * kHid + kOutMax, *isg = mu + kIn;
  h8 b;
  for (int j = 0; j < 8; ++j) b[j] = (_Float16)((x[j] - mu[j]) * isg[j]);
  return b;
}

// Outputs for NG x 16 samples (groups G0 .. G0 + NG - 1 of a wave's 64): in
// group G, lanes 0..15 hold the standardised inputs of sample 16 G + lane
// (zeros elsewhere).  Result register r of out[G - G0] in lane l: output
// drow(l/16, r) of sample 16 G + l % 16 -- with ROT, output
// (drow(l/16, r) - 4 G) mod 16 (the rotated output layer).  The groups go
// through each layer together, so that their independent matrix core chains
// overlap the activations of the others.
template <bool ROT, int NG, int G0>
__device__ __forceinline__ void net(const Net16 &N, const h8 *rot, const float *bias, const h8 *b,
                                    f4 *out) {
  const int g = (threadIdx.x & 63) >> 4;
  h8 h[NG][2];
  f4 t[NG][4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const f4 c = bias4(bias, mt * 16, g);
#pragma unroll
    for (int G = 0; G < NG; ++G) t[G][mt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(N.a1[mt], b[G], c, 0, 0, 0);
  }
#pragma unroll
  for (int G = 0; G < NG; ++G) h[G][0] = relu_pair(t[G][0], t[G][1]), h[G][1] = relu_pair(t[G][2], t[G][3]);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const f4 c = bias4(bias, kHid + mt * 16, g);
#pragma unroll
    for (int G = 0; G < NG; ++G)
      t[G][mt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
          N.a2[mt][1], h[G][1], __builtin_amdgcn_mfma_f32_16x16x32_f16(N.a2[mt][0], h[G][0], c, 0, 0, 0),
          0, 0, 0);
  }
#pragma unroll
  for (int G = 0; G < NG; ++G) h[G][0] = relu_pair(t[G][0], t[G][1]), h[G][1] = relu_pair(t[G][2], t[G][3]);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const f4 c = bias4(bias, 2 * kHid + mt * 16, g);
#pragma unroll
    for (int G = 0; G < NG; ++G)
      t[G][mt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
          N.a3[mt][1], h[G][1], __builtin_amdgcn_mfma_f32_16x16x32_f16(N.a3[mt][0], h[G][0], c, 0, 0, 0),
          0, 0, 0);
  }
#pragma unroll
  for (int G = 0; G < NG; ++G) h[G][0] = relu_pair(t[G][0], t[G][1]), h[G][1] = relu_pair(t[G][2], t[G][3]);
  if constexpr (!ROT) {
    const f4 c = bias4(bias, 3 * kHid, g);
#pragma unroll
    for (int G = 0; G < NG; ++G)
      out[G] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
          N.a4[1], h[G][1], __builtin_amdgcn_mfma_f32_16x16x32_f16(N.a4[0], h[G][0], c, 0, 0, 0), 0, 0, 0);
  } else {
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int G = 0; G < NG; ++G) {
      // rows 4 g + r of group G0 + G hold output (4 (g - G0 - G) + r) mod 16
      const f4 c = *reinterpret_cast<const f4 *>(bias + 3 * kHid + ((4 * (g - G0 - G)) & 15));
      const h8 w0 = rot[(2 * (G0 + G)) * 64 + l];
      const h8 w1 = rot[(2 * (G0 + G) + 1) * 64 + l];
      out[G] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
          w1, h[G][1], __builtin_amdgcn_mfma_f32_16x16x32_f16(w0, h[G][0], c, 0, 0, 0), 0, 0, 0);
    }
  }
}

// Generic inference over stored inputs x[n][8] -> y[n][n_out].
__global__ __launch_bounds__(kThreads, 2) void k_mlp_infer16(int n_out, const h8 *__restrict__ packed,
                                                          int64_t n, const float *__restrict__ x,
                                                          float *__restrict__ y) {
  __shared__ __attribute__((aligned(16))) float bias[kBiasFloats];
  Net16 N;
  load_net(packed, &N, bias);
  __syncthreads();
  const int l = threadIdx.x & 63, g = l >> 4;
  const int64_t nwaves = (int64_t)gridDim.x * (kThreads / kWave);
  const int64_t w0 = (int64_t)blockIdx.x * (kThreads / kWave) + threadIdx.x / kWave;
  for (int64_t s0 = w0 * 64; s0 < n; s0 += nwaves * 64) {
    h8 b[4];
    for (int G = 0; G < 4; ++G) {
      const int64_t s = s0 + 16 * G + (l & 15);
      b[G] = (h8){0, 0, 0, 0, 0, 0, 0, 0};
      if (g == 0 && s < n) {
        float f[8];
        for (int j = 0; j < 8; ++j) f[j] = x[s * kIn + j];
        b[G] = standardise(f, bias);
      }
    }
    f4 out[4];
    net<false, 2, 0>(N, nullptr, bias, b, out);
    net<false, 2, 2>(N, nullptr, bias, b + 2, out + 2);
    for (int G = 0; G < 4; ++G) {
      const int64_t s = s0 + 16 * G + (l & 15);
      for (int r = 0; r < 4; ++r) {
        const int o = drow(g, r);
        if (s < n && o < n_out) y[s * n_out + o] = out[G][r];
      }
    }
  }
}

// ------------------------------------------------------------ pair inputs
// Per-triangle part of the inputs: centroid c = v0 + (2 e1 + e2) / 3 and
// unit normal (FP64), longest edge d, area and aspect sqrt(3)/4 d^2 / area
// (FP32).
struct TriIn {
  double c[3], n[3];
  float d, area, aspect;
};

__device__ __forceinline__ TriIn tri_inputs(const double *g, int64_t L, int i) {
  TriIn t;
  double a2 = 0, b2 = 0, s2 = 0;
  for (int k = 0; k < 3; ++k) {
    const double e1 = g[(G_E1X + k) * L + i], e2 = g[(G_E2X + k) * L + i];
    t.c[k] = g[(G_V0X + k) * L + i] + (2.0 * e1 + e2) / 3.0;
    t.n[k] = g[(G_NX + k) * L + i];
    a2 = fma(e1, e1, a2);
    b2 = fma(e2, e2, b2);
    s2 = fma(e1 + e2, e1 + e2, s2);
  }
  const double d = sqrt(fmax(a2, fmax(b2, s2)));
  const double area = 0.5 * g[G_SG * L + i];
  t.d = (float)d;
  t.area = (float)area;
  t.aspect = (float)(0.4330127018922193 * d * d / area);  // sqrt(3)/4 d^2 / area
  return t;
}

// Larger / smaller of two non-negative floats by their bit patterns (which
// order like integers), without the NaN quieting of fmaxf / fminf.
__device__ __forceinline__ float nonneg_max(float a, float b) {
  return __int_as_float(max(__float_as_int(a), __float_as_int(b)));
}
__device__ __forceinline__ float nonneg_min(float a, float b) {
  return __int_as_float(min(__float_as_int(a), __float_as_int(b)));
}
// ln x for a normal x > 0 (v_log_f32 gives log2).
__device__ __forceinline__ float ln_normal(float x) {
  return 0.69314718055994531f * __builtin_amdgcn_logf(x);
}

// Inputs of the pair (i, j): x0 = ln(r / D), x1, x2 aspects, x3 area ratio,
// x4 = kappa D, x5 = ln max(|n_i - n_j|^2, 1e-12), x6 = layer,
// x7 = ln max(|<c_i - c_j, n_j>| / r, 1e-8).  Differences in FP64, the rest
// in FP32: ratios by v_rcp_f32 / v_rsq_f32, logarithms of ratios (no
// cancellation), x0 as ln(r^2 / D^2) / 2.
__device__ __forceinline__ void pair_inputs(const TriIn &ti, const TriIn &tj, int layer,
                                            float kappa, float f[8]) {
  const double s0 = ti.c[0] - tj.c[0], s1 = ti.c[1] - tj.c[1], s2 = ti.c[2] - tj.c[2];
  const double m0 = ti.n[0] - tj.n[0], m1 = ti.n[1] - tj.n[1], m2 = ti.n[2] - tj.n[2];
  const float r2 = (float)fma(s0, s0, fma(s1, s1, s2 * s2));
  const float dn = (float)fabs(fma(s0, tj.n[0], fma(s1, tj.n[1], s2 * tj.n[2])));
  const float nn = (float)fma(m0, m0, fma(m1, m1, m2 * m2));
  const float D = nonneg_max(ti.d, tj.d);
  f[0] = 0.5f * ln_normal(r2 * __builtin_amdgcn_rcpf(D * D));
  f[1] = ti.aspect;
  f[2] = tj.aspect;
  f[3] = nonneg_min(ti.area, tj.area) * __builtin_amdgcn_rcpf(nonneg_max(ti.area, tj.area));
  f[4] = kappa * D;
  f[5] = ln_normal(nonneg_max(nn, 1e-12f));
  f[6] = (float)layer;
  f[7] = ln_normal(nonneg_max(dn * __builtin_amdgcn_rsqf(r2), 1e-8f));
}

// Per-triangle inputs of a mesh, structure of arrays with leading dimension
// ldt: c[3][ldt], n[3][ldt] (FP64), d, area, aspect [3][ldt] (FP32).
__global__ void k_tri_inputs(const double *__restrict__ geo, int64_t L, int nt,
                             double *__restrict__ tc, double *__restrict__ tn,
                             float *__restrict__ tf, int64_t ldt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nt) return;
  const TriIn t = tri_inputs(geo, L, i);
  for (int m = 0; m < 3; ++m) tc[m * ldt + i] = t.c[m], tn[m * ldt + i] = t.n[m];
  tf[i] = t.d;
  tf[ldt + i] = t.area;
  tf[2 * ldt + i] = t.aspect;
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
  const TriIn ti = tri_inputs(a.geo, a.ldg, i), tj = tri_inputs(a.geo, a.ldg, j);
  float f[8];
  pair_inputs(ti, tj, LAYER, (float)a.kappa, f);
  for (int c = 0; c < kIn; ++c) a.x[k * kIn + c] = f[c];
  const Acc<KERNEL> ref = regular_pair_fp64<KERNEL, LAYER>(a.geo, a.ldg, a.rule[kSelQ], a.nq[kSelQ],
                                                          a.kappa, i, j);
  // size of a single-layer entry of the pair: |tau_i| |tau_j| / (4 pi r)
  double r2 = 0.0;
  for (int c = 0; c < 3; ++c) r2 = fma(ti.c[c] - tj.c[c], ti.c[c] - tj.c[c], r2);
  const double s = 0.25 * a.geo[G_SG * a.ldg + i] * a.geo[G_SG * a.ldg + j] * kInv4Pi / sqrt(r2);
  const double den = fmax(entry_abs<KERNEL>(ref), 1e-3 * s);
  for (int q = 0; q < kSelQ; ++q) {
    const Acc<KERNEL> v = regular_pair_fp64<KERNEL, LAYER>(a.geo, a.ldg, a.rule[q], a.nq[q],
                                                          a.kappa, i, j);
    a.t[k * kSelQ + q] = (float)log10(fmax(entry_abs_diff<KERNEL, LAYER>(v, ref) / den, 1e-16));
  }
}

// Orders of the entries of near-field blocks: 0 for pairs with a common
// vertex, else the smallest order in [q_min, q_plain - 1] whose predicted
// error plus the margin is at most log10(tol) at it and at every order above
// it below q_plain; q_plain when q_plain - 1 fails.  One workgroup per block,
// 64 x 64 sub-tiles; the sub-tile's triangles' inputs are staged in LDS, each
// lane forms the inputs of one group of a.group rows of a column (one entry
// for a.group = 1), and each wave runs the network on its 64 groups in four
// sets of 16 (inputs moved to lanes 0..15 by lane shuffles).
constexpr int kSelTile = 64;

__global__ __launch_bounds__(kThreads, 2) void k_select_orders(const SelectArgs a) {
  __shared__ __attribute__((aligned(16))) float bias[kBiasFloats];
  __shared__ double sc[2][3][kSelTile], sn[2][3][kSelTile];
  __shared__ float sd[2][3][kSelTile];  // d, area, aspect
  __shared__ int sv[2][3][kSelTile], sbad;
  __shared__ h8 srot[8 * 64];  // the rotated output layer (slots kRotSlot ..)
  __shared__ float srange[16];  // training range of the inputs: minima, maxima
  const int tid = threadIdx.x;
  Net16 N;
  load_net(reinterpret_cast<const h8 *>(a.net), &N, bias);
  if (tid < 16) srange[tid] = a.range ? a.range[tid] : (tid < 8 ? -INFINITY : INFINITY);
  for (int k = tid; k < 8 * 64; k += kThreads) srot[k] = reinterpret_cast<const h8 *>(a.net)[kRotSlot * 64 + k];
  const int l = tid & 63, g = l >> 4, wave = tid / kWave;
  const float kappa = (float)a.kappa;
  const int64_t T = a.ldt;
  for (int b = blockIdx.x; b < a.nblocks; b += gridDim.x) {
  const int64_t rp0 = a.row_ptr[b], rp1 = a.row_ptr[b + 1];
  const int64_t cp0 = a.col_ptr[b], cp1 = a.col_ptr[b + 1];
  const int64_t off = a.out_off[b];
  bool ok = rp0 >= 0 && rp0 <= rp1 && rp1 <= a.row_len && cp0 >= 0 && cp0 <= cp1 &&
            cp1 <= a.col_len && off >= 0 && off <= a.out_len;
  const int64_t nr = rp1 - rp0, nc = cp1 - cp0;
  ok = ok && (nr == 0 || nc <= (a.out_len - off) / nr);
  if (!ok) {
    if (tid == 0) atomicOr(a.flags, FLAG_EINVAL);
    continue;  // uniform
  }
  for (int64_t r0 = 0; r0 < nr; r0 += kSelTile)
    for (int64_t c0 = 0; c0 < nc; c0 += kSelTile) {
      const int tr = (int)min((int64_t)kSelTile, nr - r0), tc = (int)min((int64_t)kSelTile, nc - c0);
      __syncthreads();  // LDS of the previous sub-tile no longer read
      if (tid == 0) sbad = 0;
      __syncthreads();
      for (int k = tid; k < tr + tc; k += kThreads) {
        const int side = k < tr ? 0 : 1, p = side ? k - tr : k;
        const int id = side ? a.col_idx[cp0 + c0 + p] : a.row_idx[rp0 + r0 + p];
        if (id < 0 || id >= a.nt) {
          sbad = 1;
          continue;
        }
        for (int m = 0; m < 3; ++m) {
          sc[side][m][p] = a.tin_c[m * T + id];
          sn[side][m][p] = a.tin_n[m * T + id];
          sv[side][m][p] = a.tri[3 * (int64_t)id + m];
          sd[side][m][p] = a.tin_f[m * T + id];
        }
      }
      __syncthreads();
      if (sbad) {
        if (tid == 0) atomicOr(a.flags, FLAG_EINVAL);
        continue;  // uniform
      }
      // a lane takes a group of G rows of one column (G = a.group, 1 .. 8):
      // the network runs once for the group, on the inputs of its pair with
      // the smallest distance over diameter (the one its error grows with
      // most) and the largest row aspect of the group
      const int G = a.group, ngr = (tr + G - 1) / G;
      const int ne = ngr * tc;
      // e / ngr by a float reciprocal: e < 4096 and ngr <= 64 keep
      // (e + 1/2) / ngr at least 1 / 128 away from an integer, far above the
      // rounding error
      const float itr = 1.0f / (float)ngr;
      for (int e0 = wave * 64; e0 < ne; e0 += kThreads) {  // no barrier inside: trip counts differ
        const int e = e0 + l;
        const bool live = e < ne;
        const int cq = (int)(((float)e + 0.5f) * itr);
        const int rg = live ? (e - cq * ngr) * G : 0, cl = live ? cq : 0;
        const int rn = live ? min(G, tr - rg) : 0;  // rows of this group
        unsigned cls_bits = 0;  // 2 bits per row: the pair class
        int rep = -1;
        float best = 0.0f, aspect = 0.0f;
        for (int u = 0; u < rn; ++u) {
          const int rl = rg + u;
          const int cls = shared_vertex_count(sv[0][0][rl], sv[0][1][rl], sv[0][2][rl],
                                              sv[1][0][cl], sv[1][1][cl], sv[1][2][cl]);
          cls_bits |= (unsigned)cls << (2 * u);
          if (cls) continue;
          double r2 = 0.0;
          for (int m = 0; m < 3; ++m) {
            const double d = sc[0][m][rl] - sc[1][m][cl];
            r2 = fma(d, d, r2);
          }
          const float D = nonneg_max(sd[0][0][rl], sd[1][0][cl]);
          const float ratio = (float)r2 * __builtin_amdgcn_rcpf(D * D);
          if (rep < 0 || ratio < best) best = ratio, rep = rl;
          aspect = nonneg_max(aspect, sd[0][2][rl]);
        }
        // standardised inputs of this lane's group, packed as four half2 words
        uint32_t w[4] = {0, 0, 0, 0};
        bool outside = false;
        if (rep >= 0) {
          TriIn ti, tj;
          for (int m = 0; m < 3; ++m) {
            ti.c[m] = sc[0][m][rep], ti.n[m] = sn[0][m][rep];
            tj.c[m] = sc[1][m][cl], tj.n[m] = sn[1][m][cl];
          }
          ti.d = sd[0][0][rep], ti.area = sd[0][1][rep], ti.aspect = aspect;
          tj.d = sd[1][0][cl], tj.area = sd[1][1][cl], tj.aspect = sd[1][2][cl];
          float f[8];
          pair_inputs(ti, tj, a.layer, kappa, f);
          // an input outside the training range (or not a number) keeps the
          // plain order: the network is not trusted where it was not trained
          for (int k = 0; k < 8; ++k) outside = outside || !(f[k] >= srange[k] && f[k] <= srange[8 + k]);
          const h8 hb = standardise(f, bias);
          for (int k = 0; k < 4; ++k) {
            const _Float16 lo = hb[2 * k], hi = hb[2 * k + 1];
            w[k] = (uint32_t)__builtin_bit_cast(uint16_t, lo) |
                   ((uint32_t)__builtin_bit_cast(uint16_t, hi) << 16);
          }
        }
        // group G of the network: every lane takes the inputs of entry
        // 16 G + l % 16; only lanes 0..15 meet nonzero first-layer weights
        // (the other lanes' k-slots multiply zeros, exactly)
        h8 bop[4];
        for (int Gn = 0; Gn < 4; ++Gn) {
          uint32_t v[4];
          for (int k = 0; k < 4; ++k) v[k] = (uint32_t)__shfl((int)w[k], Gn * 16 + (l & 15), kWave);
          bop[Gn] = __builtin_bit_cast(h8, v);
        }
        f4 out[4];
        net<true, 2, 0>(N, srot, bias, bop, out);
        net<true, 2, 2>(N, srot, bias, bop + 2, out + 2);
        // This lane's entry is sample l % 16 of group g: its outputs 0..3 are
        // out[g][0..3] here, output 4 is out[g][0] of lane l + 16 (mod 64).
        // Only outputs q_min - 1 .. q_plain - 2 are needed (uniform).
        float pred[5];
#pragma unroll
        for (int o = 0; o < 4; ++o) {
          pred[o] = 0.0f;
          if (o >= a.q_min - 1 && o <= a.q_plain - 2)
            pred[o] = g == 0 ? out[0][o] : g == 1 ? out[1][o] : g == 2 ? out[2][o] : out[3][o];
        }
        pred[4] = 0.0f;
        if (a.q_plain >= 6) {  // the next lane group's copy for group g - 1
          const int gs = (g + 3) & 3;
          const float v = gs == 0 ? out[0][0] : gs == 1 ? out[1][0] : gs == 2 ? out[2][0] : out[3][0];
          pred[4] = __shfl(v, (l + 16) & 63, kWave);
        }
        // t = q_plain - 1 down to q_min while e_t + margin <= log10 tol
        int q = a.q_plain;
        bool run = true;
#pragma unroll
        for (int t = kSelQ - 1; t >= 1; --t) {
          if (t <= a.q_plain - 1 && t >= a.q_min) {  // uniform
            run = run && pred[t - 1] + a.margin <= a.log_tol;
            q = run ? t : q;
          }
        }
        if (outside) q = a.q_plain;
        for (int u = 0; u < rn; ++u) {
          const int cls = (cls_bits >> (2 * u)) & 3;
          a.orders[off + (r0 + rg + u) + nr * (c0 + cl)] = (int8_t)(cls ? 0 : q);
        }
      }
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

size_t mlp_packed_bytes() { return sizeof(h8) * kNetSlots * 64 + sizeof(float) * kBiasFloats; }

hipError_t launch_pack_net(int n_out, const float *P, void *packed, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_net, dim3(1), dim3(64), 0, s, n_out, P, static_cast<h8 *>(packed));
  return hipGetLastError();
}

hipError_t launch_tri_inputs(const double *geo, int64_t ldg, int nt, double *tc, double *tn,
                             float *tf, int64_t ldt, hipStream_t s) {
  if (nt == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tri_inputs, dim3((nt + 255) / 256), dim3(256), 0, s, geo, ldg, nt, tc, tn,
                     tf, ldt);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(bool f16, int n_out, const float *P, const void *packed, int64_t n,
                              const float *x, float *y, hipStream_t s) {
  if (f16) {
    const int64_t waves = (n + 63) / 64;  // 64 samples per wave and step
    const unsigned grid = (unsigned)std::min<int64_t>((waves + 3) / 4, 2048);
    hipLaunchKernelGGL(k_mlp_infer16, dim3(grid), dim3(kThreads), 0, s, n_out,
                       static_cast<const h8 *>(packed), n, x, y);
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

hipError_t launch_select_orders(const SelectArgs &a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_select_orders, dim3(std::min(a.nblocks, grid)), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace bem
