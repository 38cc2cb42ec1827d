// Learned surrogate of the moment -> transmittance reconstruction: a
// 7 -> 64 -> 64 -> 1 MLP (tanh-GELU hidden layers, sigmoid output F, optical
// depth m_0 F) with bf16 weights and activations and fp32 accumulation.
//
// Every layer is a dense contraction and runs on the matrix cores
// (v_mfma_f32_32x32x16_bf16), 64 queries per wave:
//   layer 1  Z1[64x64] = X[64x16] W1p^T,   X = (x_hi, x_lo) split of the 7 fp32
//            inputs into bf16 pairs (W1p repeats W1 for both halves), so the
//            inputs keep ~16 mantissa bits;
//   layer 2  Z2[64x64] = H1[64x64] W2^T,   H1 = bf16(GELU(Z1 + b1));
//   layer 3  out = GELU(Z2 + b2) . w3 + b3, reduced through LDS;
// and the training step adds dW2 = dZ2^T H1, dH1 = dZ2 W2, dW1 = dZ1^T X on
// the same instruction. MFMA operand layout (wave64, 32x32x16): lane l holds
// A[l % 32][8 (l / 32) + e] and B[8 (l / 32) + e][l % 32], e = 0..7, and
// accumulator element r of lane l is C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
#include "kernels.h"

namespace mb {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kH = 64;       // hidden width
constexpr int kIn = 7;       // inputs: 6 moment features + query
constexpr int kXStride = 16; // bf16 per input row (hi 0..6, lo 7..13, 0 pad)
// flat fp32 parameter vector theta
constexpr int O_W1 = 0;              // [64][7]
constexpr int O_B1 = O_W1 + kH * kIn; // [64]
constexpr int O_W2 = O_B1 + kH;       // [64][64] (out, in)
constexpr int O_B2 = O_W2 + kH * kH;  // [64]
constexpr int O_W3 = O_B2 + kH;       // [64]
constexpr int O_B3 = O_W3 + kH;       // [1]
constexpr int kParams = O_B3 + 1;     // 4737
// per-wave gradient partial layout (dW1 kept unfolded over the hi/lo halves)
constexpr int Q_W1 = 0;               // [64][16]
constexpr int Q_B1 = Q_W1 + kH * 16;
constexpr int Q_W2 = Q_B1 + kH;
constexpr int Q_B2 = Q_W2 + kH * kH;
constexpr int Q_W3 = Q_B2 + kH;
constexpr int Q_B3 = Q_W3 + kH;
constexpr int Q_LOSS = Q_B3 + 1;
constexpr int kPartial = Q_LOSS + 3;  // padded to a multiple of 4

struct MlpPacked {
  uint16_t w1[kH][kXStride];  // bf16 [n][k]: cols 0..6 = W1, 7..13 = W1, 14..15 = 0
  uint16_t w2[kH][kH];        // bf16 [n][k]
  uint16_t w2t[kH][kH];       // bf16 [k][n]
  float w3[kH];               // bf16-rounded
  float b1[kH], b2[kH];
  float b3;
  float pad[63];
  float w1f[kIn][kH];         // bf16-rounded W1 as fp32, [k][n] (input gradient)
};
static_assert(sizeof(MlpPacked) % 16 == 0, "packed weights must be 16-byte sized");

__host__ __device__ inline uint16_t bf16_bits(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf16_float(uint16_t b) {
  uint32_t u = ((uint32_t)b) << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

__device__ __forceinline__ float gelu_d(float x, float& d) {
  // tanh form 0.5 x (1 + tanh(u)), u = c (x + a x^3), evaluated as x s with
  // s = 1 / (1 + exp(-2u)) (the same function: 0.5 (1 + tanh u) = s):
  // one exp2 and one reciprocal, no tanh
  const float c = 0.7978845608028654f, a = 0.044715f;
  const float k = -2.f * c * 1.4426950408889634f;  // -2 c log2(e)
  const float x2 = x * x;
  const float e = __builtin_amdgcn_exp2f(k * x * (1.f + a * x2));
  const float sg = fast_rcp(1.f + e);
  d = sg + 2.f * c * x * sg * (1.f - sg) * (1.f + 3.f * a * x2);
  return x * sg;
}
__device__ __forceinline__ float gelu(float x) {
  float d;
  return gelu_d(x, d);
}

__device__ __forceinline__ bf16x8 lds_bf16x8(const uint16_t* p) {
  return *reinterpret_cast<const bf16x8*>(p);
}

__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int c_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_pack(const float* th, MlpPacked* p) {
  for (int i = threadIdx.x; i < kH * kXStride; i += blockDim.x) {
    int n = i / kXStride, k = i % kXStride;
    float v = k < kIn ? th[O_W1 + n * kIn + k] : (k < 2 * kIn ? th[O_W1 + n * kIn + k - kIn] : 0.f);
    p->w1[n][k] = bf16_bits(v);
  }
  for (int i = threadIdx.x; i < kH * kH; i += blockDim.x) {
    int n = i / kH, k = i % kH;
    uint16_t b = bf16_bits(th[O_W2 + i]);
    p->w2[n][k] = b;
    p->w2t[k][n] = b;
  }
  for (int i = threadIdx.x; i < kH; i += blockDim.x) {
    p->w3[i] = bf16_float(bf16_bits(th[O_W3 + i]));
    p->b1[i] = th[O_B1 + i];
    p->b2[i] = th[O_B2 + i];
  }
  if (threadIdx.x == 0) p->b3 = th[O_B3];
  for (int i = threadIdx.x; i < 63; i += blockDim.x) p->pad[i] = 0.f;
  for (int i = threadIdx.x; i < kH * kIn; i += blockDim.x) {
    int n = i / kIn, k = i % kIn;
    p->w1f[k][n] = bf16_float(bf16_bits(th[O_W1 + i]));
  }
}

// LDS working sets of one wave. The layer-3 row sums reuse the H1 (or dZ2)
// storage once the matrix-core reads of it are complete (barrier between).
struct FwdLds {
  uint16_t x[64][kXStride];  // inputs, hi/lo bf16
  union {
    uint16_t h1[64][kH + 8];  // H1 [q][k] (rows padded against bank conflicts)
    float s[64][33];          // layer-3 partial sums [q][column]
  };
};
struct TrainLds {
  uint16_t x[64][kXStride];
  uint16_t xt[32][64 + 8];   // X^T [k][q], rows 16..31 zero
  uint16_t h1[64][kH + 8];
  uint16_t h1t[kH][64 + 8];  // H1^T [k][q]
  union {
    uint16_t dz[64][kH + 8];  // dZ2 [q][n]
    float s[64][33];
  };
  uint16_t dzt[kH][64 + 8];  // dZ2^T [n][q], later dZ1^T
  float dout[64];
};

// stage the wave's 64 input vectors (v: this lane's kIn inputs) as bf16 pairs
template <class L>
__device__ __forceinline__ void stage_inputs(L& w, const float* v, int lane) {
  uint16_t hi[kIn], lo[kIn];
#pragma unroll
  for (int k = 0; k < kIn; ++k) {
    hi[k] = bf16_bits(v[k]);
    lo[k] = bf16_bits(v[k] - bf16_float(hi[k]));
  }
#pragma unroll
  for (int k = 0; k < kXStride; ++k) {
    uint16_t b = k < kIn ? hi[k] : (k < 2 * kIn ? lo[k - kIn] : (uint16_t)0);
    w.x[lane][k] = b;
    if constexpr (sizeof(L) == sizeof(TrainLds)) w.xt[k][lane] = b;
  }
  if constexpr (sizeof(L) == sizeof(TrainLds))
#pragma unroll
    for (int k = kXStride; k < 32; ++k) w.xt[k][lane] = 0;
}

template <class L>
__device__ __forceinline__ void load_inputs(L& w, const float* x, int64_t q, bool valid, int lane, float& m0) {
  float v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = valid ? x[q * 8 + k] : 0.f;
  m0 = v[7];
  stage_inputs(w, v, lane);
}

// layers 1-3 for the wave's 64 queries; returns the output pre-activation of
// query `lane` and leaves the Z1/Z2 tiles (and H1, H1^T) for the backward pass
template <class L>
__device__ __forceinline__ float mlp_forward_wave(L& w, const MlpPacked& P, int lane, f32x16 z1[2][2],
                                                  f32x16 z2[2][2]) {
  constexpr bool kTrain = sizeof(L) == sizeof(TrainLds);
  const int lr = lane & 31, hk = 8 * (lane >> 5);
  // layer 1
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      f32x16 acc = {};
      acc = mfma(lds_bf16x8(&w.x[32 * mt + lr][hk]), lds_bf16x8(&P.w1[32 * nt + lr][hk]), acc);
      z1[mt][nt] = acc;
    }
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      int n = 32 * nt + lr;
      float b = P.b1[n];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        int q = 32 * mt + c_row(r, lane);
        float zz = z1[mt][nt][r] + b;
        z1[mt][nt][r] = zz;
        uint16_t hb = bf16_bits(gelu(zz));
        w.h1[q][n] = hb;
        if constexpr (kTrain) w.h1t[n][q] = hb;
      }
    }
  __syncthreads();
  // layer 2
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      f32x16 acc = {};
#pragma unroll
      for (int kt = 0; kt < 4; ++kt)
        acc = mfma(lds_bf16x8(&w.h1[32 * mt + lr][16 * kt + hk]), lds_bf16x8(&P.w2[32 * nt + lr][16 * kt + hk]), acc);
      z2[mt][nt] = acc;
    }
  __syncthreads();
  // layer 3: per-lane partial sums over its two columns, reduced through LDS
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      float s = 0.f;
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        int n = 32 * nt + lr;
        float zz = z2[mt][nt][r] + P.b2[n];
        z2[mt][nt][r] = zz;
        s += gelu(zz) * P.w3[n];
      }
      w.s[32 * mt + c_row(r, lane)][lr] = s;
    }
  }
  __syncthreads();
  float out = P.b3;
#pragma unroll
  for (int c = 0; c < 32; ++c) out += w.s[lane][c];
  __syncthreads();
  return out;
}

__device__ __forceinline__ float sigmoid(float x) { return fast_rcp(1.f + __expf(-x)); }

__global__ __launch_bounds__(256) void k_mlp_forward(const MlpPacked* gp, const float* x, int64_t n, float* f_out) {
  __shared__ MlpPacked P;
  __shared__ FwdLds ws[4];
  {
    const float4* src = reinterpret_cast<const float4*>(gp);
    float4* dst = reinterpret_cast<float4*>(&P);
    for (int i = threadIdx.x; i < (int)(sizeof(MlpPacked) / 16); i += blockDim.x) dst[i] = src[i];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  FwdLds& w = ws[wave];
  const int64_t chunks = (n + 63) / 64;
  const int64_t per_block = ((chunks + gridDim.x - 1) / gridDim.x + 3) / 4 * 4;  // uniform per block
  for (int64_t it = 0; it < per_block; it += 4) {
    int64_t chunk = (int64_t)blockIdx.x * per_block + it + wave;
    int64_t q = chunk * 64 + lane;
    bool valid = q < n;
    float m0;
    load_inputs(w, x, q, valid, lane, m0);
    __syncthreads();
    f32x16 z1[2][2], z2[2][2];
    float out = mlp_forward_wave(w, P, lane, z1, z2);
    if (valid) f_out[q] = sigmoid(out);
  }
}

// The same network on the render's query list: the inputs of query i are the
// six features of pixel q_pix[i] and the standardised query q_z[i]. The
// number of queries is read on the device (the render pass appends them).
__global__ __launch_bounds__(256) void k_mlp_forward_gather(const MlpPacked* gp, const float* pixfeat, const int* q_pix,
                                                            const float* q_z, const unsigned long long* q_count,
                                                            int64_t q_cap, int64_t n_pix, float* f_out) {
  __shared__ MlpPacked P;
  __shared__ FwdLds ws[4];
  const unsigned long long cnt = *q_count;
  const int64_t n = cnt < (unsigned long long)q_cap ? (int64_t)cnt : q_cap;
  if (n == 0) return;
  {
    const float4* src = reinterpret_cast<const float4*>(gp);
    float4* dst = reinterpret_cast<float4*>(&P);
    for (int i = threadIdx.x; i < (int)(sizeof(MlpPacked) / 16); i += blockDim.x) dst[i] = src[i];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  FwdLds& w = ws[wave];
  const int64_t chunks = (n + 63) / 64;
  const int64_t per_block = ((chunks + gridDim.x - 1) / gridDim.x + 3) / 4 * 4;
  for (int64_t it = 0; it < per_block; it += 4) {
    int64_t q = ((int64_t)blockIdx.x * per_block + it + wave) * 64 + lane;
    bool valid = q < n;
    float v[kIn];
    // slots of a list that overflowed may hold no query: keep their pixel
    // index inside the image (their outputs are never read)
    int64_t p = valid ? (int64_t)q_pix[q] : 0;
    p = (p >= 0 && p < n_pix) ? p : 0;
    const float* pf = pixfeat + (size_t)p * kPixFeat;
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = valid ? pf[k] : 0.f;
    v[6] = valid ? q_z[q] : 0.f;
    stage_inputs(w, v, lane);
    __syncthreads();
    f32x16 z1[2][2], z2[2][2];
    float out = mlp_forward_wave(w, P, lane, z1, z2);
    if (valid) f_out[q] = sigmoid(out);
  }
}

// The network at the nodes of every pixel's table (the tabulated schedule):
// entry q = p * n_nodes + g takes the six features of pixel p and the
// standardised query z_g = -kTabZ + g 2 kTabZ / (n_nodes - 1).
__global__ __launch_bounds__(256) void k_mlp_table(const MlpPacked* gp, const float* pixfeat, int64_t n_pix,
                                                   int n_nodes, float* tab) {
  __shared__ MlpPacked P;
  __shared__ FwdLds ws[4];
  const int64_t n = n_pix * n_nodes;
  {
    const float4* src = reinterpret_cast<const float4*>(gp);
    float4* dst = reinterpret_cast<float4*>(&P);
    for (int i = threadIdx.x; i < (int)(sizeof(MlpPacked) / 16); i += blockDim.x) dst[i] = src[i];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  FwdLds& w = ws[wave];
  const float dz = 2.f * kTabZ / (float)(n_nodes - 1);
  const int64_t chunks = (n + 63) / 64;
  const int64_t per_block = ((chunks + gridDim.x - 1) / gridDim.x + 3) / 4 * 4;
  for (int64_t it = 0; it < per_block; it += 4) {
    const int64_t q = ((int64_t)blockIdx.x * per_block + it + wave) * 64 + lane;
    const bool valid = q < n;
    const int64_t p = valid ? q / n_nodes : 0;
    const int g = valid ? (int)(q - p * n_nodes) : 0;
    const float* pf = pixfeat + (size_t)p * kPixFeat;
    float v[kIn];
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = valid ? pf[k] : 0.f;
    v[6] = -kTabZ + dz * (float)g;
    stage_inputs(w, v, lane);
    __syncthreads();
    f32x16 z1[2][2], z2[2][2];
    float out = mlp_forward_wave(w, P, lane, z1, z2);
    if (valid) tab[q] = sigmoid(out);
  }
}

// F and its gradient dF/dx with respect to the 7 inputs for every query of
// the render's list (for the backward pass through the surrogate): the
// forward pass as above, then dZ2 = F (1 - F) w3 GELU'(Z2) (bf16) on the
// matrix cores against W2, dZ1 = dH1 GELU'(Z1) (bf16, staged by rows) and
// dx = dZ1 W1 on the vector unit. Two waves per workgroup; the H1 storage is
// reused for dZ2 and then dZ1. out: [cap][8] = F, dF/dx_0..6.
struct GradInLds {
  uint16_t x[64][kXStride];
  union {
    uint16_t h1[64][kH + 8];
    float s[64][33];
    uint16_t dz[64][kH + 8];
  };
  float dout[64];
};

__global__ __launch_bounds__(128) void k_mlp_input_grad_gather(const MlpPacked* gp, const float* pixfeat,
                                                               const int* q_pix, const float* q_z,
                                                               const unsigned long long* q_count, int64_t q_cap,
                                                               int64_t n_pix, float* out_g) {
  __shared__ MlpPacked P;
  __shared__ GradInLds ws[2];
  const unsigned long long cnt = *q_count;
  const int64_t n = cnt < (unsigned long long)q_cap ? (int64_t)cnt : q_cap;
  if (n == 0) return;
  {
    const float4* src = reinterpret_cast<const float4*>(gp);
    float4* dst = reinterpret_cast<float4*>(&P);
    for (int i = threadIdx.x; i < (int)(sizeof(MlpPacked) / 16); i += blockDim.x) dst[i] = src[i];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 31, hk = 8 * (lane >> 5);
  GradInLds& w = ws[wave];
  const int64_t chunks = (n + 63) / 64;
  const int64_t per_block = ((chunks + gridDim.x - 1) / gridDim.x + 1) / 2 * 2;
  for (int64_t it = 0; it < per_block; it += 2) {
    int64_t q = ((int64_t)blockIdx.x * per_block + it + wave) * 64 + lane;
    bool valid = q < n;
    float v[kIn];
    int64_t p = valid ? (int64_t)q_pix[q] : 0;
    p = (p >= 0 && p < n_pix) ? p : 0;
    const float* pf = pixfeat + (size_t)p * kPixFeat;
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = valid ? pf[k] : 0.f;
    v[6] = valid ? q_z[q] : 0.f;
    stage_inputs(w, v, lane);
    __syncthreads();
    f32x16 z1[2][2], z2[2][2];
    float out = mlp_forward_wave(w, P, lane, z1, z2);
    const float f = sigmoid(out);
    w.dout[lane] = f * (1.f - f);
    __syncthreads();
    // dZ2 = dF/dout w3 GELU'(Z2), bf16, rows [q][n]
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        int n2 = 32 * nt + lr;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          int qq = 32 * mt + c_row(r, lane);
          float d;
          gelu_d(z2[mt][nt][r], d);
          w.dz[qq][n2] = bf16_bits(w.dout[qq] * P.w3[n2] * d);
        }
      }
    __syncthreads();
    // dH1 = dZ2 W2
    f32x16 dh1[2][2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        f32x16 acc = {};
#pragma unroll
        for (int kt = 0; kt < 4; ++kt)
          acc = mfma(lds_bf16x8(&w.dz[32 * mt + lr][16 * kt + hk]), lds_bf16x8(&P.w2t[32 * nt + lr][16 * kt + hk]),
                     acc);
        dh1[mt][nt] = acc;
      }
    __syncthreads();
    // dZ1 = dH1 GELU'(Z1), bf16, rows [q][n]
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        int n1 = 32 * nt + lr;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          int qq = 32 * mt + c_row(r, lane);
          float d;
          gelu_d(z1[mt][nt][r], d);
          w.dz[qq][n1] = bf16_bits(dh1[mt][nt][r] * d);
        }
      }
    __syncthreads();
    // dx_k = sum_n dZ1[q][n] W1[n][k] for this lane's query
    float g[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) g[k] = 0.f;
#pragma unroll
    for (int n8 = 0; n8 < kH; n8 += 8) {
      bf16x8 row = lds_bf16x8(&w.dz[lane][n8]);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float dzv = (float)row[e];
#pragma unroll
        for (int k = 0; k < kIn; ++k) g[k] += dzv * P.w1f[k][n8 + e];
      }
    }
    if (valid) {
      float* o = out_g + q * 8;
      o[0] = f;
#pragma unroll
      for (int k = 0; k < kIn; ++k) o[1 + k] = g[k];
    }
    __syncthreads();
  }
}

// Forward + backward of the loss mean_q (exp(-m0_q F_q) - T_q)^2 over the
// batch; one gradient partial per wave (deterministic reduction afterwards).
constexpr int kTrainWaves = 2;

__global__ __launch_bounds__(128) void k_mlp_train(const MlpPacked* gp, const float* x, const float* t_target,
                                                   int64_t n, float* partials) {
  __shared__ MlpPacked P;
  __shared__ TrainLds ws[kTrainWaves];
  {
    const float4* src = reinterpret_cast<const float4*>(gp);
    float4* dst = reinterpret_cast<float4*>(&P);
    for (int i = threadIdx.x; i < (int)(sizeof(MlpPacked) / 16); i += blockDim.x) dst[i] = src[i];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 31, hk = 8 * (lane >> 5);
  TrainLds& w = ws[wave];
  f32x16 gw2[2][2], gw1[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    gw1[a] = f32x16{};
#pragma unroll
    for (int b = 0; b < 2; ++b) gw2[a][b] = f32x16{};
  }
  float gb1[2] = {0.f, 0.f}, gb2[2] = {0.f, 0.f}, gw3[2] = {0.f, 0.f}, gb3 = 0.f, loss = 0.f;
  const float inv_n = 1.f / (float)n;
  const int64_t chunks = (n + 63) / 64;
  const int64_t per_block =
      ((chunks + gridDim.x - 1) / gridDim.x + kTrainWaves - 1) / kTrainWaves * kTrainWaves;
  for (int64_t it = 0; it < per_block; it += kTrainWaves) {
    int64_t chunk = (int64_t)blockIdx.x * per_block + it + wave;
    int64_t q = chunk * 64 + lane;
    bool valid = q < n;
    float m0;
    load_inputs(w, x, q, valid, lane, m0);
    __syncthreads();
    f32x16 z1[2][2], z2[2][2];
    float out = mlp_forward_wave(w, P, lane, z1, z2);
    // loss and d loss / d out for query `lane`
    float f = sigmoid(out);
    float tp = __expf(-m0 * f);
    float diff = valid ? tp - t_target[q] : 0.f;
    loss += diff * diff;
    float dout = valid ? 2.f * diff * inv_n * (-m0 * tp) * f * (1.f - f) : 0.f;
    w.dout[lane] = dout;
    gb3 += dout;
    __syncthreads();
    // dZ2 = dout w3 GELU'(Z2); accumulate dw3, db2; stage dZ2 (bf16) both ways
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        int n2 = 32 * nt + lr;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          int qq = 32 * mt + c_row(r, lane);
          float d;
          float a2 = gelu_d(z2[mt][nt][r], d);
          float dq = w.dout[qq];
          gw3[nt] += a2 * dq;
          float dz2 = dq * P.w3[n2] * d;
          gb2[nt] += dz2;
          uint16_t b = bf16_bits(dz2);
          w.dz[qq][n2] = b;
          w.dzt[n2][qq] = b;
        }
      }
    __syncthreads();
    // dW2 += dZ2^T H1 ; dH1 = dZ2 W2
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int kt = 0; kt < 4; ++kt)
          gw2[mt][nt] = mfma(lds_bf16x8(&w.dzt[32 * mt + lr][16 * kt + hk]),
                             lds_bf16x8(&w.h1t[32 * nt + lr][16 * kt + hk]), gw2[mt][nt]);
    f32x16 dh1[2][2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        f32x16 acc = {};
#pragma unroll
        for (int kt = 0; kt < 4; ++kt)
          acc = mfma(lds_bf16x8(&w.dz[32 * mt + lr][16 * kt + hk]), lds_bf16x8(&P.w2t[32 * nt + lr][16 * kt + hk]),
                     acc);
        dh1[mt][nt] = acc;
      }
    __syncthreads();
    // dZ1 = dH1 GELU'(Z1); db1; stage dZ1^T (bf16)
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        int n1 = 32 * nt + lr;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          int qq = 32 * mt + c_row(r, lane);
          float d;
          gelu_d(z1[mt][nt][r], d);
          float dz1 = dh1[mt][nt][r] * d;
          gb1[nt] += dz1;
          w.dzt[n1][qq] = bf16_bits(dz1);
        }
      }
    __syncthreads();
    // dW1 (unfolded over the 16 input slots) += dZ1^T X
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int kt = 0; kt < 4; ++kt)
        gw1[mt] = mfma(lds_bf16x8(&w.dzt[32 * mt + lr][16 * kt + hk]), lds_bf16x8(&w.xt[lr][16 * kt + hk]), gw1[mt]);
    __syncthreads();
  }
  // write this wave's partial gradient
  float* out = partials + ((size_t)blockIdx.x * kTrainWaves + wave) * kPartial;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      int row = 32 * mt + c_row(r, lane);
      if (lr < kXStride) out[Q_W1 + row * kXStride + lr] = gw1[mt][r];
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) out[Q_W2 + row * kH + 32 * nt + lr] = gw2[mt][nt][r];
    }
  // per-lane vectors: lanes l and l^32 hold the two row halves of a column
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    float a = gb1[nt] + __shfl_xor(gb1[nt], 32, 64);
    float b = gb2[nt] + __shfl_xor(gb2[nt], 32, 64);
    float c = gw3[nt] + __shfl_xor(gw3[nt], 32, 64);
    if (lane < 32) {
      out[Q_B1 + 32 * nt + lr] = a;
      out[Q_B2 + 32 * nt + lr] = b;
      out[Q_W3 + 32 * nt + lr] = c;
    }
  }
  float sb3 = gb3, sl = loss;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    sb3 += __shfl_xor(sb3, m, 64);
    sl += __shfl_xor(sl, m, 64);
  }
  if (lane == 0) {
    out[Q_B3] = sb3;
    out[Q_LOSS] = sl;
  }
}

// Sum the per-wave partials in a fixed order and fold dW1's hi/lo halves.
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* partials, int n_waves, int64_t n, float* grad,
                                                    float* loss) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kParams) return;
  auto sum_at = [&](int qi) {
    float s = 0.f;
    for (int w = 0; w < n_waves; ++w) s += partials[(size_t)w * kPartial + qi];
    return s;
  };
  if (p == kParams) {
    if (loss) *loss = sum_at(Q_LOSS) / (float)n;
    return;
  }
  float g;
  if (p < O_B1) {
    int nn = p / kIn, k = p % kIn;
    g = sum_at(Q_W1 + nn * kXStride + k) + sum_at(Q_W1 + nn * kXStride + k + kIn);
  } else if (p < O_W2) {
    g = sum_at(Q_B1 + p - O_B1);
  } else if (p < O_B2) {
    g = sum_at(Q_W2 + p - O_W2);
  } else if (p < O_W3) {
    g = sum_at(Q_B2 + p - O_B2);
  } else if (p < O_B3) {
    g = sum_at(Q_W3 + p - O_W3);
  } else {
    g = sum_at(Q_B3);
  }
  grad[p] = g;
}

__global__ __launch_bounds__(256) void k_adam(float* th, float* m, float* v, const float* g, int64_t count, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  float gi = g[i];
  float mi = b1 * m[i] + (1.f - b1) * gi;
  float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------
int mlp_param_count() { return kParams; }
size_t mlp_packed_bytes() { return sizeof(MlpPacked); }

static int mlp_grid(int64_t n, int waves) {
  int64_t chunks = (n + 63) / 64;
  int64_t blocks = (chunks + waves - 1) / waves;
  return (int)(blocks < 1024 ? (blocks < 1 ? 1 : blocks) : 1024);
}

size_t mlp_workspace_bytes(int64_t n) { return (size_t)mlp_grid(n, kTrainWaves) * kTrainWaves * kPartial * sizeof(float); }

hipError_t launch_mlp_pack(const float* theta, void* packed, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_pack, dim3(1), dim3(256), 0, s, theta, (MlpPacked*)packed);
  return hipGetLastError();
}

hipError_t launch_mlp_forward_gather(const void* packed, const float* pixfeat, int64_t n_pix, const int* q_pix,
                                     const float* q_z, const unsigned long long* q_count, int64_t q_cap, float* f,
                                     hipStream_t s) {
  if (q_cap <= 0 || n_pix <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_forward_gather, dim3(mlp_grid(q_cap, 4)), dim3(256), 0, s, (const MlpPacked*)packed,
                     pixfeat, q_pix, q_z, q_count, q_cap, n_pix, f);
  return hipGetLastError();
}

hipError_t launch_mlp_table(const void* packed, const float* pixfeat, int64_t n_pix, int n_nodes, float* tab,
                            hipStream_t s) {
  if (n_pix <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_table, dim3(mlp_grid(n_pix * n_nodes, 4)), dim3(256), 0, s, (const MlpPacked*)packed,
                     pixfeat, n_pix, n_nodes, tab);
  return hipGetLastError();
}

hipError_t launch_mlp_input_grad_gather(const void* packed, const float* pixfeat, int64_t n_pix, const int* q_pix,
                                        const float* q_z, const unsigned long long* q_count, int64_t q_cap,
                                        float* out_g, hipStream_t s) {
  if (q_cap <= 0 || n_pix <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_input_grad_gather, dim3(mlp_grid(q_cap, 2)), dim3(128), 0, s, (const MlpPacked*)packed,
                     pixfeat, q_pix, q_z, q_count, q_cap, n_pix, out_g);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const void* packed, const float* x, int64_t n, float* f, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_forward, dim3(mlp_grid(n, 4)), dim3(256), 0, s, (const MlpPacked*)packed, x, n, f);
  return hipGetLastError();
}

hipError_t launch_mlp_loss_grad(const void* packed, const float* x, const float* t, int64_t n, float* grad,
                                float* loss, float* ws, hipStream_t s) {
  int grid = mlp_grid(n, kTrainWaves);
  hipLaunchKernelGGL(k_mlp_train, dim3(grid), dim3(128), 0, s, (const MlpPacked*)packed, x, t, n, ws);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kParams + 1 + 255) / 256), dim3(256), 0, s, ws, grid * kTrainWaves, n,
                     grad, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* th, float* m, float* v, const float* g, int64_t count, int step, float lr, float b1,
                       float b2, float eps, hipStream_t s) {
  float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, th, m, v, g, count, lr, b1, b2,
                     eps, c1, c2);
  return hipGetLastError();
}

}  // namespace mb
