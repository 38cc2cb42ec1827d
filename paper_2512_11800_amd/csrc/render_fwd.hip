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
#include "kernels.h"
#include "recon.h"

namespace mb {

struct Stage {
  float4 f[kRecF4][kBlock];
};

struct RayG {
  float mu, sig, omega;
};

__device__ __forceinline__ int remap_xcd(int bid, int nblocks) {
  // blocks are dispatched round-robin over the 8 XCDs; give each XCD a
  // contiguous run of tiles so neighbouring tiles share its L2
  int per = nblocks >> 3;
  return (bid & 7) * per + (bid >> 3);
}

__device__ __forceinline__ void load_batch(Stage& st, const float4* rec, const int* sorted_rec, int b, int nb) {
  int tid = threadIdx.x;
  if (tid < nb) {
    const float4* src = rec + (size_t)sorted_rec[b + tid] * kRecF4;
#pragma unroll
    for (int k = 0; k < kRecF4; ++k) st.f[k][tid] = src[k];
  }
}

__device__ __forceinline__ bool covers(const Stage& st, int j, float u, float v, bool inside, float& dx,
                                       float& dy) {
  float4 f0 = st.f[0][j], f1 = st.f[1][j];
  dx = u - f0.x;
  dy = v - f0.y;
  float ax = dx - f0.z, ay = dy - f0.w;
  float c1 = ax * f1.x + ay * f1.y;
  float c2 = -ax * f1.y + ay * f1.x;
  return inside && fabsf(c1) <= f1.z && fabsf(c2) <= f1.w;
}

// Eqs. 4-6 for the pixel ray in the projected-mean frame (see common.h)
__device__ __forceinline__ RayG ray_params(const Stage& st, int j, float dx, float dy, float lam) {
  float4 f2 = st.f[2][j], f3 = st.f[3][j], f4 = st.f[4][j];
  float w = st.f[5][j].x;
  float d = f2.x + 2.f * (f2.y * dx + f2.z * dy) + f2.w * dx * dx + 2.f * f3.x * dx * dy + f3.y * dy * dy;
  float e = f3.z + f3.w * dx + f4.x * dy;
  float x = f4.y * dx * dx + 2.f * f4.z * dx * dy + f4.w * dy * dy;
  float id = fast_rcp(d);
  RayG g;
  g.mu = lam * e * id;
  g.sig = lam * fast_rsq(d);
  g.omega = w * expf(-0.5f * x * id);
  return g;
}

// warped moments of one ray Gaussian, Eqs. 10-12 (t_f -> inf), in the pixel's
// moment variable; the boundary term enters with '+' (App. C)
template <int K>
__device__ __forceinline__ void particle_moments(const RayG& g, const PixelBasis& pb, float tn, float* m) {
  float mus = fmaxf(g.mu, tn);
  float ys = warp_y(pb, mus, mus - pb.tc);
  float yp = warp_dy(pb, mus);
  float gg = ys + yp * (g.mu - mus);
  float is = fast_rcp(g.sig);
  float bn = (tn - g.mu) * kInvSqrt2 * is;
  float e = expf(-bn * bn);
  float s2 = g.sig * g.sig;
  m[0] = g.omega * g.sig * kSqrtHalfPi * erfcf(bn);
  float bnd = yp * g.omega * s2 * e;
  m[1] = gg * m[0] + bnd;
  float un = gg + yp * (tn - g.mu);
  float unp = un;
  float v2 = yp * yp * s2;
#pragma unroll
  for (int k = 2; k <= K; ++k) {
    m[k] = gg * m[k - 1] + (float)(k - 1) * v2 * m[k - 2] + bnd * unp;
    unp *= un;
  }
}

__device__ __forceinline__ float phi_fn(float x) {
  // (1 - e^-x) / x, continued by its series near 0
  return fabsf(x) < 1e-4f ? 1.f - x * (0.5f - x * (1.f / 6.f)) : -expm1f(-x) / x;
}

// Quadrature of Eq. 7 for one Gaussian against the pixel's bounds; returns q.
template <int NH, int NQ>
__device__ __forceinline__ float particle_quadrature(const RayG& g, const PixelBasis& pb, const LInv<NH>& L,
                                                     float m0, float tn, const RenderArgs& a) {
  float tau[NQ], off[NQ], sj[NQ];
  bool cl[NQ];
  float dtc = g.mu - pb.tc;
#pragma unroll
  for (int j = 0; j < NQ; ++j) {
    off[j] = a.kappa * g.sig * a.xq[j];
    float t = g.mu + off[j];
    cl[j] = t < tn;
    float dt = cl[j] ? (tn - pb.tc) : (dtc + off[j]);
    t = cl[j] ? tn : t;
    float y = warp_y(pb, t, dt);
    tau[j] = m0 * bound_F<NH>(L, y, a.beta);
    float r = (t - g.mu) * fast_rcp(g.sig);
    sj[j] = g.omega * (cl[j] ? expf(-0.5f * r * r) : a.eq[j]);
  }
  float q = 0.f;
#pragma unroll
  for (int j = 0; j + 1 < NQ; ++j) {
    float delta = cl[j + 1] ? 0.f : (cl[j] ? (g.mu + off[j + 1] - tn) : (off[j + 1] - off[j]));
    q += expf(-tau[j]) * delta * phi_fn(tau[j + 1] - tau[j]) * sj[j];
  }
  return q;
}

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
  LInv<NH> L;
  bool fallback = false;
  if (acc[0] > 0.0) {
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
      bool cov = covers(st, j, u, v, inside, dx, dy);
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
