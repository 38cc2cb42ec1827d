// Forward render: one workgroup per 16x16 tile (one thread per pixel, each
// wave an 8x8 quadrant). The tile's Gaussian list is streamed through LDS in
// batches of 256 records, three times:
//   pass 0  the pixel's moment variable (mean and spread of its depth mass),
//   pass 1  warped power moments, Eqs. 10-12, summed in double (Moment pass),
//   setup   Cholesky of the Hankel matrix, kept as L^-1 (Sec. 3.2),
//   pass 2  per-Gaussian quadrature, Eq. 7 / App. B, against the bounds
//           (Quadrature pass), accumulating sum q_i (r, g, b, 1),
//   epilogue  Eq. 15 rescaling (Rescale pass).
// A wave skips a Gaussian when none of its 64 pixels is covered (ballot).
#include "render_common.h"

namespace mb {

template <int K, int NQ>
__global__ __launch_bounds__(256) void k_render_fwd(RenderArgs a, CamSet cams) {
  constexpr int NH = K / 2;
  __shared__ Stage st;
  const int tiles_per_cam = a.tiles_x * a.tiles_y;
  const int n_keys = tiles_per_cam * a.n_cams;
  const int key = remap_xcd(blockIdx.x, gridDim.x);
  if (key >= n_keys) return;
  const int ci = key / tiles_per_cam;
  const int tile = key - ci * tiles_per_cam;
  const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
  const CamConst& c = cams.c[ci];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int px = tx * kTile + (wave & 1) * 8 + (lane & 7);
  const int py = ty * kTile + (wave >> 1) * 8 + (lane >> 3);
  const bool inside = px < c.width && py < c.height;
  const float u = (float)px + 0.5f, v = (float)py + 0.5f;
  const float rx = (u - c.cx) / c.fx, ry = (v - c.cy) / c.fy;
  const float lam = sqrtf(1.f + rx * rx + ry * ry);
  const float tn = c.tn;
  const int2 rg = a.ranges[key];

  // ---- pass 0: the pixel's moment variable ---------------------------------
  float wsum = 0.f, mean = 0.f, m2 = 0.f;
  for (int b = rg.x; b < rg.y; b += kBlock) {
    int nb = min(kBlock, rg.y - b);
    __syncthreads();
    load_batch(st, a.rec, a.sorted_rec, b, nb);
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
      float dx, dy;
      bool cov = covers(st, j, u, v, inside, dx, dy);
      if (__ballot(cov) == 0) continue;
      if (cov) {
        RayG g = ray_params(st, j, dx, dy, lam);
        float wgt = g.omega * g.sig;
        if (wgt > 0.f) {
          wsum += wgt;
          float d = g.mu - mean;
          mean += d * wgt / wsum;
          m2 += wgt * (d * (g.mu - mean) + g.sig * g.sig);
        }
      }
    }
  }
  float tc = fmaxf(mean, tn);
  float sd = wsum > 0.f ? sqrtf(fmaxf(m2 / wsum, 0.f)) : 1.f;
  {
    float q = 1.f + 0.8f * tc, xn = 1.f + 0.8f * tn;
    float gp = 1.2f * xn * sqrtf(xn) / (q * q * sqrtf(q));  // g_hat'(tc)
    sd = fmaxf(sd * gp, 1e-30f);
  }
  const PixelBasis pb = make_basis(tc, sd, tn);

  // ---- pass 1: moments ------------------------------------------------------
  double acc[K + 1];
#pragma unroll
  for (int k = 0; k <= K; ++k) acc[k] = 0.0;
  for (int b = rg.x; b < rg.y; b += kBlock) {
    int nb = min(kBlock, rg.y - b);
    __syncthreads();
    load_batch(st, a.rec, a.sorted_rec, b, nb);
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
      float dx, dy;
      bool cov = covers(st, j, u, v, inside, dx, dy);
      if (__ballot(cov) == 0) continue;
      if (cov) {
        RayG g = ray_params(st, j, dx, dy, lam);
        float m[K + 1];
        particle_moments<K>(g, pb, tn, m);
#pragma unroll
        for (int k = 0; k <= K; ++k) acc[k] += (double)m[k];
      }
    }
  }

  // ---- per-pixel setup ------------------------------------------------------
  const float m0 = (float)acc[0];
  // a pixel whose optical depth is below kMinDepth is empty: its radiance
  // (about m0 times a colour) is negligible, and its moment vector is too close
  // to the float32 underflow range to define a measure
  const bool live = acc[0] > kMinDepth;
  LInv<NH> L;
  bool fallback = false;
  if (live) {
    double bn[K + 1];
    bn[0] = 1.0;
#pragma unroll
    for (int k = 1; k <= K; ++k) bn[k] = acc[k] / acc[0];
    fallback = !hankel_factor<NH>(bn, L);
  } else {
#pragma unroll
    for (int i = 0; i < (NH + 1) * (NH + 2) / 2; ++i) L.l[i] = 0.f;
  }

  // ---- pass 2: quadrature ---------------------------------------------------
  float sr = 0.f, sg = 0.f, sb = 0.f, so = 0.f;
  int n_cov = 0;
  for (int b = rg.x; b < rg.y; b += kBlock) {
    int nb = min(kBlock, rg.y - b);
    __syncthreads();
    load_batch(st, a.rec, a.sorted_rec, b, nb);
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
      float dx, dy;
      bool cov = covers(st, j, u, v, inside && live, dx, dy);
      if (__ballot(cov) == 0) continue;
      if (cov) {
        RayG g = ray_params(st, j, dx, dy, lam);
        float q = particle_quadrature<NH, NQ>(g, pb, L, m0, tn, a);
        ++n_cov;
        float4 f5 = st.f[5][j];
        sr += q * f5.y;
        sg += q * f5.z;
        sb += q * f5.w;
        so += q;
      }
    }
  }

  // ---- epilogue: Eq. 15 ------------------------------------------------------
  if (!inside) return;
  float alpha = -expm1f(-m0);
  float tr = expf(-m0);
  float inv_o = 1.f / fmaxf(a.eps, so);
  size_t pix = ((size_t)ci * c.height + py) * c.width + px;
  float* out = a.image + pix * 3;
  out[0] = alpha * sr * inv_o + tr * c.bg[0];
  out[1] = alpha * sg * inv_o + tr * c.bg[1];
  out[2] = alpha * sb * inv_o + tr * c.bg[2];
  float4* sv = reinterpret_cast<float4*>(a.saved + pix * MB_SAVED_FLOATS_PER_PIXEL);
  sv[0] = make_float4(sr, sg, sb, so);
  // covering count; stored as -(count + 1) when the Hankel factor needed a fallback
  sv[1] = make_float4(tc, sd, m0, fallback ? -(float)(n_cov + 1) : (float)n_cov);
}

hipError_t launch_render_forward(const RenderArgs& a, const CamSet& cams, int n_moments, int n_intervals,
                                 hipStream_t s) {
  int n_keys = a.tiles_x * a.tiles_y * a.n_cams;
  int nblocks = ((n_keys + 7) / 8) * 8;
  dim3 grid(nblocks), block(kBlock);
#define MB_LAUNCH(KK, NN)                                                           \
  if (n_moments == KK && n_intervals == NN) {                                       \
    hipLaunchKernelGGL((k_render_fwd<KK, NN + 1>), grid, block, 0, s, a, cams);     \
    return hipGetLastError();                                                       \
  }
  MB_LAUNCH(4, 3)
  MB_LAUNCH(6, 3)
  MB_LAUNCH(4, 5)
  MB_LAUNCH(6, 5)
#undef MB_LAUNCH
  return hipErrorInvalidValue;
}

}  // namespace mb
