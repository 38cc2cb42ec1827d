// Device-side building blocks shared by the kernels of the rendering path.
//
// Geometry follows the paper's ray-space formulation (Eqs. 4-6, App. A) but is
// evaluated in a form that stays accurate in float32: every ray through a
// pixel is written relative to the ray through the Gaussian's projected mean,
// d_un = mean_c / mean_c.z + J delta (delta = pixel offset from the projected
// mean, J = diag(1/fx, 1/fy, 0)). With B = S^-1 R^T (camera frame),
// mu_g = B mean_c and G = B J:
//   d_g . d_g  = D(delta) = |mu_g/z|^2 + 2 (G^T mu_g / z) . delta + delta^T G^T G delta
//   mu_g . d_g = E(delta) = |mu_g|^2 / z + (G^T mu_g) . delta
//   |o_g x d_g|^2 = X(delta) = delta^T P^T P delta,  P = [mu_g]_x G
// (mu_g x mu_g = 0 removes the large cancelling terms of Eq. 6), so for the
// unit ray of length-lambda = |d_un|:
//   mu = lambda E / D,  Sigma = lambda / sqrt(D),  K = -X / (2 D)   (Eqs. 4-6).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mb3dgs.h"

namespace mb {

constexpr int kTile = 16;
constexpr int kBlock = 256;
constexpr int kRecF4 = 6;  // one render record = 6 float4
// records sit 8 float4 apart in memory: each fills one 128-byte line, so a
// gathered record costs one line instead of straddling two
constexpr int kRecStride = 8;
constexpr float kPi = 3.14159265358979323846f;
constexpr float kSqrtHalfPi = 1.2533141373155003f;  // sqrt(pi/2)
constexpr float kInvSqrt2 = 0.7071067811865476f;
constexpr double kMinDepth = 1e-20;  // optical depth below which a pixel is empty
// surrogate: per-pixel record (6 features, m0, basis centre, basis scale,
// covering count, mean and standard deviation of the normalised measure in
// the moment variable) and harvested training sample (6 features, query, m0,
// transmittance, selection hash bits, pixel index, record * (N+1) + edge)
constexpr int kPixFeat = 12;
// tabulated schedule: the reconstruction per pixel at equally spaced nodes of
// the standardised query on [-kTabZ, kTabZ], linearly interpolated
constexpr float kTabZ = 4.f;
constexpr int kTabMaxNodes = 256;
constexpr int kMaxMoments = 8;  // highest moment order K supported
// Heavy tiles (more list entries than kSplitEntries) are rendered by four
// workgroups, one per 8x8 quadrant, whose four waves share the quadrant's
// pixels and take every fourth list entry. The decision depends on the tile's
// own list only, so a camera renders the same alone or in a batch. The grid
// has room for every tile to split; unused blocks exit at once.
constexpr int kSplitEntries = 512;
__host__ __device__ inline int render_blocks(int n_keys) { return 4 * n_keys; }
constexpr int kHarvestStride = 12;

// Render record fields (float index inside the 24-float record).
enum RecField {
  R_P0X = 0, R_P0Y, R_RCX, R_RCY, R_E1X, R_E1Y, R_H1, R_H2,
  R_D0, R_D1X, R_D1Y, R_D2XX, R_D2XY, R_D2YY, R_E0, R_EX,
  R_EY, R_XXX, R_XXY, R_XYY, R_W, R_CR, R_CG, R_CB,
  R_COUNT
};

// Per-pair gradient slot fields (backward partials, one per list entry).
enum GradField {
  G_D0 = 0, G_D1X, G_D1Y, G_D2XX, G_D2XY, G_D2YY, G_E0, G_EX, G_EY,
  G_XXX, G_XXY, G_XYY, G_P0X, G_P0Y, G_W, G_CR, G_CG, G_CB,
  G_COUNT
};
constexpr int kGradStride = 20;  // floats per partial slot (padded to 80 B)

struct CamConst {
  float r[9];  // world-to-camera rotation, row-major
  float t[3];
  float o[3];  // camera origin in world coordinates
  float fx, fy, cx, cy, tn;
  float bg[3];
  int width, height;
};

struct CamSet {
  int n_cams;
  CamConst c[MB_MAX_CAMERAS];
};

// e^(-x / 2), the constant folded into one multiply before the exp2
__device__ __forceinline__ float exp_neg_half(float x) {
  return __builtin_amdgcn_exp2f(-0.72134752044448170f * x);  // -log2(e) / 2
}

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Copy rows [0, nrows) of kPer contiguous floats (nrows <= NT) between global
// memory and LDS rows of kRow floats with NT threads, coalesced. Each thread
// issues all its loads before any store: a loop with a runtime bound would
// wait on every load in turn.
template <int kPer, int kRow, int NT>
__device__ __forceinline__ void stage_rows(float* lds, const float* src, int nrows) {
  const int cnt = nrows * kPer;
  float v[kPer];
#pragma unroll
  for (int it = 0; it < kPer; ++it) {
    const int i = it * NT + (int)threadIdx.x;
    v[it] = i < cnt ? src[i] : 0.f;
  }
#pragma unroll
  for (int it = 0; it < kPer; ++it) {
    const int i = it * NT + (int)threadIdx.x;
    if (i < cnt) lds[(i / kPer) * kRow + i % kPer] = v[it];
  }
}
template <int kPer, int kRow, int NT>
__device__ __forceinline__ void unstage_rows(float* dst, const float* lds, int nrows) {
  const int cnt = nrows * kPer;
  constexpr int kChunk = 8;  // LDS reads in flight per thread (bounds the registers)
  // an opaque copy of the thread index: otherwise the compiler hoists every
  // address of the unrolled loop to the kernel's start, where they stay live
  int tid = (int)threadIdx.x;
  asm volatile("" : "+v"(tid));
#pragma unroll
  for (int c0 = 0; c0 < kPer; c0 += kChunk) {
    float v[kChunk];
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      const int i = (c0 + k) * NT + tid;
      v[k] = (c0 + k < kPer && i < cnt) ? lds[(i / kPer) * kRow + i % kPer] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      const int i = (c0 + k) * NT + tid;
      if (c0 + k < kPer && i < cnt) dst[i] = v[k];
    }
  }
}

// erfc with an exact shortcut: for b < -3.9, erfc(b) = 2 - erfc(-b) with
// erfc(-b) < 4e-8, below half an ulp of 2, so the float result is 2 exactly.
// Most ray Gaussians lie far beyond the near plane (b << 0) and skip erfcf.
__device__ __forceinline__ float erfc_fast(float b) {
  if (b < -3.9f) return 2.f;
  return erfcf(b);
}

// ---------------------------------------------------------------------------
// Minimal forward-mode dual number (one tangent) for the per-Gaussian chain
// rule of the backward pass: the same templated code computes the record
// coefficients in float (forward) and their directional derivatives (backward).
// ---------------------------------------------------------------------------
struct Dual {
  float v, d;
  __host__ __device__ Dual() : v(0.f), d(0.f) {}
  __host__ __device__ Dual(float x) : v(x), d(0.f) {}
  __host__ __device__ Dual(float x, float dx) : v(x), d(dx) {}
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__device__ __forceinline__ Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
  float r = a.v / b.v;
  return Dual(r, (a.d - r * b.d) / b.v);
}
__device__ __forceinline__ Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
__device__ __forceinline__ Dual dsqrt(Dual a) { float s = sqrtf(a.v); return Dual(s, a.d * 0.5f / s); }
__device__ __forceinline__ float dsqrt(float a) { return sqrtf(a); }
__device__ __forceinline__ double dsqrt(double a) { return sqrt(a); }
__device__ __forceinline__ float val(float a) { return a; }
__device__ __forceinline__ float val(Dual a) { return a.v; }

// ---------------------------------------------------------------------------
// Per (camera, Gaussian) ray-space coefficients, templated on the arithmetic
// type (the preprocess evaluates them in double).
// ---------------------------------------------------------------------------
template <class T>
struct Coefs {
  T p0x, p0y;              // projected mean (pixels)
  T D0, D1x, D1y, D2xx, D2xy, D2yy;
  T E0, Ex, Ey;
  T Xxx, Xxy, Xyy;
  T mug[3];                // B mean_c
  T muc[3];                // mean in camera coordinates
};

template <class T>
__device__ __forceinline__ void compute_coefs(const T mean[3], const T scale[3], const T quat[4],
                                              const CamConst& c, Coefs<T>& o) {
  // rotation of the Gaussian from its normalised quaternion (w, x, y, z)
  T qn = dsqrt(quat[0] * quat[0] + quat[1] * quat[1] + quat[2] * quat[2] + quat[3] * quat[3]);
  T w = quat[0] / qn, x = quat[1] / qn, y = quat[2] / qn, z = quat[3] / qn;
  T rq[9];
  rq[0] = T(1.f) - T(2.f) * (y * y + z * z); rq[1] = T(2.f) * (x * y - w * z); rq[2] = T(2.f) * (x * z + w * y);
  rq[3] = T(2.f) * (x * y + w * z); rq[4] = T(1.f) - T(2.f) * (x * x + z * z); rq[5] = T(2.f) * (y * z - w * x);
  rq[6] = T(2.f) * (x * z - w * y); rq[7] = T(2.f) * (y * z + w * x); rq[8] = T(1.f) - T(2.f) * (x * x + y * y);
  // camera-frame rotation R_c = R_wc R_q and mean
  T rc[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      rc[i * 3 + j] = T(c.r[i * 3 + 0]) * rq[0 * 3 + j] + T(c.r[i * 3 + 1]) * rq[1 * 3 + j] +
                      T(c.r[i * 3 + 2]) * rq[2 * 3 + j];
#pragma unroll
  for (int i = 0; i < 3; ++i)
    o.muc[i] = T(c.r[i * 3 + 0]) * mean[0] + T(c.r[i * 3 + 1]) * mean[1] + T(c.r[i * 3 + 2]) * mean[2] +
               T(c.t[i]);
  // B = S^-1 R_c^T: row k of B is column k of R_c divided by scale_k
  T b[9];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T inv = T(1.f) / scale[k];
    b[k * 3 + 0] = rc[0 * 3 + k] * inv;
    b[k * 3 + 1] = rc[1 * 3 + k] * inv;
    b[k * 3 + 2] = rc[2 * 3 + k] * inv;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k)
    o.mug[k] = b[k * 3 + 0] * o.muc[0] + b[k * 3 + 1] * o.muc[1] + b[k * 3 + 2] * o.muc[2];
  T iz = T(1.f) / o.muc[2];
  o.p0x = T(c.cx) + T(c.fx) * o.muc[0] * iz;
  o.p0y = T(c.cy) + T(c.fy) * o.muc[1] * iz;
  // G = B J: columns B[:,0]/fx and B[:,1]/fy
  T gx[3], gy[3], g0[3];
  T ifx = T(1.f) / T(c.fx), ify = T(1.f) / T(c.fy);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    gx[k] = b[k * 3 + 0] * ifx;
    gy[k] = b[k * 3 + 1] * ify;
    g0[k] = o.mug[k] * iz;
  }
  o.D0 = g0[0] * g0[0] + g0[1] * g0[1] + g0[2] * g0[2];
  o.D1x = gx[0] * g0[0] + gx[1] * g0[1] + gx[2] * g0[2];
  o.D1y = gy[0] * g0[0] + gy[1] * g0[1] + gy[2] * g0[2];
  o.D2xx = gx[0] * gx[0] + gx[1] * gx[1] + gx[2] * gx[2];
  o.D2xy = gx[0] * gy[0] + gx[1] * gy[1] + gx[2] * gy[2];
  o.D2yy = gy[0] * gy[0] + gy[1] * gy[1] + gy[2] * gy[2];
  T quad = o.mug[0] * o.mug[0] + o.mug[1] * o.mug[1] + o.mug[2] * o.mug[2];
  o.E0 = quad * iz;
  o.Ex = gx[0] * o.mug[0] + gx[1] * o.mug[1] + gx[2] * o.mug[2];
  o.Ey = gy[0] * o.mug[0] + gy[1] * o.mug[1] + gy[2] * o.mug[2];
  // P = [mu_g]_x G
  T px[3], py[3];
  px[0] = o.mug[1] * gx[2] - o.mug[2] * gx[1];
  px[1] = o.mug[2] * gx[0] - o.mug[0] * gx[2];
  px[2] = o.mug[0] * gx[1] - o.mug[1] * gx[0];
  py[0] = o.mug[1] * gy[2] - o.mug[2] * gy[1];
  py[1] = o.mug[2] * gy[0] - o.mug[0] * gy[2];
  py[2] = o.mug[0] * gy[1] - o.mug[1] * gy[0];
  o.Xxx = px[0] * px[0] + px[1] * px[1] + px[2] * px[2];
  o.Xxy = px[0] * py[0] + px[1] * py[1] + px[2] * py[2];
  o.Xyy = py[0] * py[0] + py[1] * py[1] + py[2] * py[2];
}

// ---------------------------------------------------------------------------
// Real spherical harmonics up to degree 3 (index l^2 + l + m), the standard
// real basis: Y_00 = 1/(2 sqrt(pi)); Y_1m = sqrt(3/(4pi)) (y, z, x); ...
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void sh_basis(T x, T y, T z, int degree, T* out) {
  out[0] = T(0.28209479177387814f);  // 1/(2 sqrt(pi))
  if (degree < 1) return;
  const float c1 = 0.4886025119029199f;  // sqrt(3/(4 pi))
  out[1] = T(c1) * y; out[2] = T(c1) * z; out[3] = T(c1) * x;
  if (degree < 2) return;
  T xx = x * x, yy = y * y, zz = z * z;
  out[4] = T(1.0925484305920792f) * x * y;              // sqrt(15/pi)/2
  out[5] = T(1.0925484305920792f) * y * z;
  out[6] = T(0.31539156525252005f) * (T(3.f) * zz - T(1.f));  // sqrt(5/pi)/4
  out[7] = T(1.0925484305920792f) * x * z;
  out[8] = T(0.5462742152960396f) * (xx - yy);           // sqrt(15/pi)/4
  if (degree < 3) return;
  out[9] = T(0.5900435899266435f) * y * (T(3.f) * xx - yy);   // sqrt(35/(2pi))/4
  out[10] = T(2.890611442640554f) * x * y * z;                 // sqrt(105/pi)/2
  out[11] = T(0.4570457994644658f) * y * (T(5.f) * zz - T(1.f));  // sqrt(21/(2pi))/4
  out[12] = T(0.3731763325901154f) * z * (T(5.f) * zz - T(3.f));  // sqrt(7/pi)/4
  out[13] = T(0.4570457994644658f) * x * (T(5.f) * zz - T(1.f));
  out[14] = T(1.445305721320277f) * z * (xx - yy);             // sqrt(105/pi)/4
  out[15] = T(0.5900435899266435f) * x * (xx - T(3.f) * yy);
}

// ---------------------------------------------------------------------------
// Depth warp with lambda = -1.5 (Sec. 3.2): g_hat(t) = 1 - ((1+0.8t)/(1+0.8t_n))^-1.5.
// Differences are taken exactly: with p = 1 + 0.8 t_c, q = 1 + 0.8 t,
//   p^-1.5 - q^-1.5 = (q - p)(q^2 + q p + p^2) / ((q^1.5 + p^1.5)(p q)^1.5),
// so y(t) = (g_hat(t) - g_hat(t_c)) / s keeps full relative precision near t_c.
// ---------------------------------------------------------------------------
struct PixelBasis {
  float tc;     // depth of the moment-variable origin
  float p;      // 1 + 0.8 tc
  float p15;    // p^1.5
  float amp;    // 0.8 (1 + 0.8 tn)^1.5 / s
};

__device__ __forceinline__ PixelBasis make_basis(float tc, float s, float tn) {
  PixelBasis b;
  b.tc = tc;
  b.p = 1.f + 0.8f * tc;
  b.p15 = b.p * sqrtf(b.p);
  float xn = 1.f + 0.8f * tn;
  b.amp = 0.8f * xn * sqrtf(xn) / s;
  return b;
}

// y at depth t, given dt = t - tc computed by the caller without cancellation
__device__ __forceinline__ float warp_y(const PixelBasis& b, float t, float dt) {
  float q = 1.f + 0.8f * t;
  float sq = fast_sqrt(q);
  float q15 = q * sq;
  float num = (q + b.p) * q + b.p * b.p;
  float den = (q15 + b.p15) * (b.p15 * q15);
  return b.amp * dt * num * fast_rcp(den);
}

// dy/dt at depth t: 1.5 amp q^-2.5
__device__ __forceinline__ float warp_dy(const PixelBasis& b, float t) {
  float q = 1.f + 0.8f * t;
  float sq = fast_sqrt(q);
  return 1.5f * b.amp * fast_rcp(q * q * sq);
}

}  // namespace mb
