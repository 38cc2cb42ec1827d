// The D-SSIM term of the training objective (Training and Densification
// paragraph: L = (1 - alpha) L1 + alpha L_D-SSIM + lambda L_consistency): the
// structural similarity of the 3DGS losses the paper extends, per colour
// channel under an 11 x 11 Gaussian window (sigma 1.5, zero padding), and its
// gradient. One workgroup per 16 x 16 tile: the tile and a 5-pixel halo are
// staged in LDS and blurred separably (rows, then columns).
//
// With a = mu_x, b = mu_y, p = E[x^2], q = E[y^2], r = E[xy] (window means)
// and S = A1 A2 / (B1 B2), A1 = 2ab + C1, A2 = 2(r - ab) + C2,
// B1 = a^2 + b^2 + C1, B2 = (p - a^2) + (q - b^2) + C2, the forward pass keeps
// dS/da, dS/dp, dS/dr per pixel and channel; the gradient of mean S with
// respect to x is then (G * dS/da + 2x G * dS/dp + y G * dS/dr) / N, G the
// (symmetric) window.
#include "kernels.h"

namespace mb {

constexpr int kSsimTile = 16;
constexpr int kSsimHalo = 5;
constexpr int kSsimIn = kSsimTile + 2 * kSsimHalo;  // 26
constexpr float kSsimC1 = 0.0001f, kSsimC2 = 0.0009f;

// separable blur of NM maps staged as in[m][26][26] -> out value at this
// thread's pixel; tmp[m][26][16] holds the row pass
template <int NM>
__device__ __forceinline__ void blur_tile(const float (*in)[kSsimIn][kSsimIn], float (*tmp)[kSsimIn][kSsimTile],
                                          const SsimArgs& a, int tid, float* out) {
  for (int e = tid; e < NM * kSsimIn * kSsimTile; e += 256) {
    const int m = e / (kSsimIn * kSsimTile), r = (e / kSsimTile) % kSsimIn, c = e % kSsimTile;
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 11; ++k) s += a.g[k] * in[m][r][c + k];
    tmp[m][r][c] = s;
  }
  __syncthreads();
  const int ty = tid / kSsimTile, tx = tid % kSsimTile;
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 11; ++k) s += a.g[k] * tmp[m][ty + k][tx];
    out[m] = s;
  }
}

__global__ __launch_bounds__(256) void k_dssim_fwd(SsimArgs a) {
  __shared__ float in[5][kSsimIn][kSsimIn];
  __shared__ float tmp[5][kSsimIn][kSsimTile];
  __shared__ float red[256];
  const int tiles_x = (a.w + kSsimTile - 1) / kSsimTile, tiles_y = (a.h + kSsimTile - 1) / kSsimTile;
  const int cam = blockIdx.x / (tiles_x * tiles_y), t = blockIdx.x % (tiles_x * tiles_y);
  const int x0 = (t % tiles_x) * kSsimTile - kSsimHalo, y0 = (t / tiles_x) * kSsimTile - kSsimHalo;
  const int tid = threadIdx.x;
  const int px = x0 + kSsimHalo + tid % kSsimTile, py = y0 + kSsimHalo + tid / kSsimTile;
  const bool inside = px < a.w && py < a.h;
  const size_t pix = ((size_t)cam * a.h + (inside ? py : 0)) * a.w + (inside ? px : 0);
  float ssum = 0.f;
  for (int ch = 0; ch < 3; ++ch) {
    __syncthreads();
    for (int e = tid; e < kSsimIn * kSsimIn; e += 256) {
      const int yy = y0 + e / kSsimIn, xx = x0 + e % kSsimIn;
      float xv = 0.f, yv = 0.f;
      if (xx >= 0 && xx < a.w && yy >= 0 && yy < a.h) {
        const size_t q = (((size_t)cam * a.h + yy) * a.w + xx) * 3 + ch;
        xv = a.image[q];
        yv = a.target[q];
      }
      in[0][e / kSsimIn][e % kSsimIn] = xv;
      in[1][e / kSsimIn][e % kSsimIn] = yv;
      in[2][e / kSsimIn][e % kSsimIn] = xv * xv;
      in[3][e / kSsimIn][e % kSsimIn] = yv * yv;
      in[4][e / kSsimIn][e % kSsimIn] = xv * yv;
    }
    __syncthreads();
    float m[5];
    blur_tile<5>(in, tmp, a, tid, m);
    const float am = m[0], bm = m[1], p = m[2], q = m[3], r = m[4];
    const float A1 = 2.f * am * bm + kSsimC1, A2 = 2.f * (r - am * bm) + kSsimC2;
    const float B1 = am * am + bm * bm + kSsimC1, B2 = (p - am * am) + (q - bm * bm) + kSsimC2;
    const float iB = 1.f / (B1 * B2);
    const float S = A1 * A2 * iB;
    if (inside) {
      ssum += S;
      if (a.coef) {
        float* c = a.coef + pix * 9 + ch * 3;
        c[0] = 2.f * bm * (A2 - A1) * iB - S * (2.f * am / B1 - 2.f * am / B2);  // dS/da
        c[1] = -S / B2;                                                        // dS/dp
        c[2] = 2.f * A1 * iB;                                                  // dS/dr
      }
    }
  }
  // fixed-order block sum of S
  red[tid] = ssum;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) a.partials[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_dssim_reduce(SsimArgs a, int nb) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) s += (double)a.partials[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *a.loss = (float)(1.0 - red[0] / ((double)a.n_cams * a.h * a.w * 3.0));
}

__global__ __launch_bounds__(256) void k_dssim_bwd(SsimArgs a) {
  __shared__ float in[3][kSsimIn][kSsimIn];
  __shared__ float tmp[3][kSsimIn][kSsimTile];
  const int tiles_x = (a.w + kSsimTile - 1) / kSsimTile, tiles_y = (a.h + kSsimTile - 1) / kSsimTile;
  const int cam = blockIdx.x / (tiles_x * tiles_y), t = blockIdx.x % (tiles_x * tiles_y);
  const int x0 = (t % tiles_x) * kSsimTile - kSsimHalo, y0 = (t / tiles_x) * kSsimTile - kSsimHalo;
  const int tid = threadIdx.x;
  const int px = x0 + kSsimHalo + tid % kSsimTile, py = y0 + kSsimHalo + tid / kSsimTile;
  const bool inside = px < a.w && py < a.h;
  const size_t pix = ((size_t)cam * a.h + (inside ? py : 0)) * a.w + (inside ? px : 0);
  // d(1 - mean S)/dx, times the caller's scale
  const float scale = -a.grad_scale / ((float)a.n_cams * (float)a.h * (float)a.w * 3.f);
  for (int ch = 0; ch < 3; ++ch) {
    __syncthreads();
    for (int e = tid; e < kSsimIn * kSsimIn; e += 256) {
      const int yy = y0 + e / kSsimIn, xx = x0 + e % kSsimIn;
      float c0 = 0.f, c1 = 0.f, c2 = 0.f;
      if (xx >= 0 && xx < a.w && yy >= 0 && yy < a.h) {
        const float* c = a.coef + (((size_t)cam * a.h + yy) * a.w + xx) * 9 + ch * 3;
        c0 = c[0];
        c1 = c[1];
        c2 = c[2];
      }
      in[0][e / kSsimIn][e % kSsimIn] = c0;
      in[1][e / kSsimIn][e % kSsimIn] = c1;
      in[2][e / kSsimIn][e % kSsimIn] = c2;
    }
    __syncthreads();
    float m[3];
    blur_tile<3>(in, tmp, a, tid, m);
    if (inside) {
      const size_t q = pix * 3 + ch;
      const float xv = a.image[q], yv = a.target[q];
      a.grad[q] += scale * (m[0] + 2.f * xv * m[1] + yv * m[2]);
    }
  }
}

hipError_t launch_dssim(const SsimArgs& a, hipStream_t s) {
  const int nb = ((a.w + kSsimTile - 1) / kSsimTile) * ((a.h + kSsimTile - 1) / kSsimTile) * a.n_cams;
  hipLaunchKernelGGL(k_dssim_fwd, dim3(nb), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_dssim_reduce, dim3(1), dim3(256), 0, s, a, nb);
  if (a.grad) hipLaunchKernelGGL(k_dssim_bwd, dim3(nb), dim3(256), 0, s, a);
  return hipGetLastError();
}

// L1 term: mean |x - y| and grad += scale sign(x - y) / n. Fixed grid, one
// double partial per block, summed in block order.
constexpr int kL1Blocks = 1024;

__global__ __launch_bounds__(256) void k_l1(const float* x, const float* y, int64_t n, float gs, float* grad,
                                            double* partials) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)kL1Blocks * 256) {
    const float d = x[i] - y[i];
    s += (double)fabsf(d);
    if (grad) grad[i] += d > 0.f ? gs : (d < 0.f ? -gs : 0.f);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_l1_reduce(const double* partials, int64_t n, float* loss) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < kL1Blocks; i += 256) s += partials[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = n > 0 ? (float)(red[0] / (double)n) : 0.f;
}

int l1_partials() { return kL1Blocks; }

hipError_t launch_l1(const float* x, const float* y, int64_t n, float grad_scale, float* loss, float* grad,
                     double* partials, hipStream_t s) {
  const float gs = n > 0 ? grad_scale / (float)n : 0.f;
  hipLaunchKernelGGL(k_l1, dim3(kL1Blocks), dim3(256), 0, s, x, y, n, gs, grad, partials);
  hipLaunchKernelGGL(k_l1_reduce, dim3(1), dim3(256), 0, s, partials, n, loss);
  return hipGetLastError();
}

int dssim_blocks(int n_cams, int w, int h) {
  return ((w + kSsimTile - 1) / kSsimTile) * ((h + kSsimTile - 1) / kSsimTile) * n_cams;
}

}  // namespace mb
