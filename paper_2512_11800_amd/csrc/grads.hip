// Per-Gaussian end of the backward pass: sum the per-(list entry, wave) slots
// of the Gradient stage over every tile and camera the Gaussian was listed
// in (its entries are contiguous, and so are a wave's), then chain the
// record-coefficient gradients to mean, scale and rotation by one reverse
// sweep through the coefficient geometry of the preprocess.
#include "kernels.h"

namespace mb {

// Sum of the four wave slots of list entry e (fixed order); a slot the
// backward pass did not write (its quadrant's coverage mask is empty) counts
// as zero.
__device__ __forceinline__ void entry_total(const float* partials, const uint8_t* used, int e, float* r) {
  const float4* sl = reinterpret_cast<const float4*>(partials + (size_t)e * 4 * kGradStride);
  const uchar4 u = reinterpret_cast<const uchar4*>(used)[e];
  const bool uw[4] = {u.x != 0, u.y != 0, u.z != 0, u.w != 0};
  float4 v[4][5];
#pragma unroll
  for (int w = 0; w < 4; ++w)
#pragma unroll
    for (int k = 0; k < 5; ++k) v[w][k] = uw[w] ? sl[w * (kGradStride / 4) + k] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const float x = ((v[0][k].x + v[1][k].x) + v[2][k].x) + v[3][k].x;
    const float y = ((v[0][k].y + v[1][k].y) + v[2][k].y) + v[3][k].y;
    const float z = ((v[0][k].z + v[1][k].z) + v[2][k].z) + v[3][k].z;
    const float t = ((v[0][k].w + v[1][k].w) + v[2][k].w) + v[3][k].w;
    if (4 * k + 0 < G_COUNT) r[4 * k + 0] = x;
    if (4 * k + 1 < G_COUNT) r[4 * k + 1] = y;
    if (4 * k + 2 < G_COUNT) r[4 * k + 2] = z;
    if (4 * k + 3 < G_COUNT) r[4 * k + 3] = t;
  }
}

constexpr int kRecRow = G_COUNT | 1;  // LDS row of one entry's total (odd: spreads banks)

__device__ __forceinline__ void cross3(const float a[3], const float b[3], float o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// Reverse-mode chain through compute_coefs: given the adjoints P of the
// record coefficients (p0, D, E, X), add d/d(mean, scale, quat) to gp[0..2],
// gp[3..5], gp[6..9]. The primal is recomputed with the same formulas; the
// sweep visits them in reverse (cross products c = a x b take
// a_bar += b x c_bar, b_bar += c_bar x a).
__device__ __forceinline__ void coefs_adjoint(const float mean[3], const float scale[3], const float quat[4],
                                              const CamConst& c, const float* P, float gp[10]) {
  // ---- primal
  const float qn = sqrtf(quat[0] * quat[0] + quat[1] * quat[1] + quat[2] * quat[2] + quat[3] * quat[3]);
  const float iq = 1.f / qn;
  const float w = quat[0] * iq, x = quat[1] * iq, y = quat[2] * iq, z = quat[3] * iq;
  float rq[9];
  rq[0] = 1.f - 2.f * (y * y + z * z); rq[1] = 2.f * (x * y - w * z); rq[2] = 2.f * (x * z + w * y);
  rq[3] = 2.f * (x * y + w * z); rq[4] = 1.f - 2.f * (x * x + z * z); rq[5] = 2.f * (y * z - w * x);
  rq[6] = 2.f * (x * z - w * y); rq[7] = 2.f * (y * z + w * x); rq[8] = 1.f - 2.f * (x * x + y * y);
  float rc[9], muc[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j)
      rc[i * 3 + j] = c.r[i * 3] * rq[j] + c.r[i * 3 + 1] * rq[3 + j] + c.r[i * 3 + 2] * rq[6 + j];
    muc[i] = c.r[i * 3] * mean[0] + c.r[i * 3 + 1] * mean[1] + c.r[i * 3 + 2] * mean[2] + c.t[i];
  }
  float is[3], b[9], mug[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    is[k] = 1.f / scale[k];
#pragma unroll
    for (int j = 0; j < 3; ++j) b[k * 3 + j] = rc[j * 3 + k] * is[k];
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) mug[k] = b[k * 3] * muc[0] + b[k * 3 + 1] * muc[1] + b[k * 3 + 2] * muc[2];
  const float iz = 1.f / muc[2];
  const float ifx = 1.f / c.fx, ify = 1.f / c.fy;
  float gx[3], gy[3], g0[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    gx[k] = b[k * 3] * ifx;
    gy[k] = b[k * 3 + 1] * ify;
    g0[k] = mug[k] * iz;
  }
  const float quad = mug[0] * mug[0] + mug[1] * mug[1] + mug[2] * mug[2];
  float px[3], py[3];
  cross3(mug, gx, px);
  cross3(mug, gy, py);
  // ---- adjoints
  float pxb[3], pyb[3], mugb[3], gxb[3], gyb[3], t[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    pxb[k] = 2.f * P[G_XXX] * px[k] + P[G_XXY] * py[k];
    pyb[k] = P[G_XXY] * px[k] + 2.f * P[G_XYY] * py[k];
  }
  cross3(gx, pxb, mugb);
  cross3(gy, pyb, t);
#pragma unroll
  for (int k = 0; k < 3; ++k) mugb[k] += t[k];
  cross3(pxb, mug, gxb);
  cross3(pyb, mug, gyb);
  float izb = P[G_E0] * quad;
  const float quadb = P[G_E0] * iz;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    gxb[k] += P[G_EX] * mug[k] + P[G_D1X] * g0[k] + 2.f * P[G_D2XX] * gx[k] + P[G_D2XY] * gy[k];
    gyb[k] += P[G_EY] * mug[k] + P[G_D1Y] * g0[k] + P[G_D2XY] * gx[k] + 2.f * P[G_D2YY] * gy[k];
    const float g0b = 2.f * P[G_D0] * g0[k] + P[G_D1X] * gx[k] + P[G_D1Y] * gy[k];
    mugb[k] += P[G_EX] * gx[k] + P[G_EY] * gy[k] + 2.f * quadb * mug[k] + g0b * iz;
    izb += g0b * mug[k];
  }
  float mucb[3] = {P[G_P0X] * c.fx * iz, P[G_P0Y] * c.fy * iz, 0.f};
  izb += P[G_P0X] * c.fx * muc[0] + P[G_P0Y] * c.fy * muc[1];
  float bb[9];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    bb[k * 3] = gxb[k] * ifx + mugb[k] * muc[0];
    bb[k * 3 + 1] = gyb[k] * ify + mugb[k] * muc[1];
    bb[k * 3 + 2] = mugb[k] * muc[2];
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) mucb[j] += mugb[0] * b[j] + mugb[1] * b[3 + j] + mugb[2] * b[6 + j];
  mucb[2] -= izb * iz * iz;
#pragma unroll
  for (int l = 0; l < 3; ++l) gp[l] += c.r[l] * mucb[0] + c.r[3 + l] * mucb[1] + c.r[6 + l] * mucb[2];
  float rcb[9];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    gp[3 + k] -= is[k] * (bb[k * 3] * b[k * 3] + bb[k * 3 + 1] * b[k * 3 + 1] + bb[k * 3 + 2] * b[k * 3 + 2]);
#pragma unroll
    for (int j = 0; j < 3; ++j) rcb[j * 3 + k] = bb[k * 3 + j] * is[k];
  }
  float R[9];  // rq_bar = R_wc^T rc_bar
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int j = 0; j < 3; ++j) R[l * 3 + j] = c.r[l] * rcb[j] + c.r[3 + l] * rcb[3 + j] + c.r[6 + l] * rcb[6 + j];
  const float wb = 2.f * (-z * R[1] + y * R[2] + z * R[3] - x * R[5] - y * R[6] + x * R[7]);
  const float xb = 2.f * (y * R[1] + z * R[2] + y * R[3] - w * R[5] + z * R[6] + w * R[7]) - 4.f * x * (R[4] + R[8]);
  const float yb = 2.f * (x * R[1] + w * R[2] + x * R[3] + z * R[5] - w * R[6] + z * R[7]) - 4.f * y * (R[0] + R[8]);
  const float zb = 2.f * (-w * R[1] + x * R[2] + w * R[3] + y * R[5] + x * R[6] + y * R[7]) - 4.f * z * (R[0] + R[4]);
  // through the normalisation n = q / |q|
  const float nd = w * wb + x * xb + y * yb + z * zb;
  gp[6] += (wb - w * nd) * iq;
  gp[7] += (xb - x * nd) * iq;
  gp[8] += (yb - y * nd) * iq;
  gp[9] += (zb - z * nd) * iq;
}

// The block's colour coefficients are staged through LDS (one padded row per
// Gaussian) so their loads and the colour-gradient stores are coalesced.
//
// Slot sums are load-balanced per wave: a wave's 64 Gaussians own one
// contiguous range of list entries per camera (the offsets are a scan over
// Gaussians), which the wave sweeps 64 entries at a time, one entry per lane,
// all loads of a window in flight together; each owner then adds its entries'
// totals from LDS in entry order. A thread walking its own entries instead
// would serialise on the largest count in its wave (several times the mean
// for the size spread of real scenes).
template <int DEG>
__global__ __launch_bounds__(128) void k_grad_finalize(GradArgs a, CamSet cams) {
  constexpr int nsh = DEG < 0 ? 1 : (DEG + 1) * (DEG + 1);
  constexpr int kPer = 3 * nsh;
  constexpr int kRow = kPer | 1;
  __shared__ float shc[128 * kRow];
  __shared__ float erec[2][64 * kRecRow];
  const int g0 = blockIdx.x * blockDim.x;
  const int nblk = min(128, a.n - g0);
  stage_rows<kPer, kRow, 128>(shc, a.colors + (size_t)g0 * kPer, nblk);
  __syncthreads();
  float* row = shc + threadIdx.x * kRow;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nw = min(64, a.n - g0 - 64 * wv);  // Gaussians of this wave (wave-uniform)
  float* rec = erec[wv];
  int g = g0 + threadIdx.x;
  if (nw > 0) {
    const bool valid = g < a.n;
    const int gl = valid ? g : g0 + 64 * wv;  // in-range index for the parameter loads
    float mean[3] = {a.means[3 * gl], a.means[3 * gl + 1], a.means[3 * gl + 2]};
    float scale[3] = {a.scales[3 * gl], a.scales[3 * gl + 1], a.scales[3 * gl + 2]};
    float quat[4] = {a.quats[4 * gl], a.quats[4 * gl + 1], a.quats[4 * gl + 2], a.quats[4 * gl + 3]};
    float gp[10];
#pragma unroll
    for (int p = 0; p < 10; ++p) gp[p] = 0.f;
    float gw = 0.f;
    float gcol[3 * nsh];
#pragma unroll
    for (int k = 0; k < 3 * nsh; ++k) gcol[k] = 0.f;

    for (int ci = 0; ci < cams.n_cams; ++ci) {
      const size_t idx = (size_t)ci * a.n + gl;
      const int cnt = valid ? a.counts[idx] : 0;
      const int off = a.offsets[idx];
      const int base = __shfl(off, 0);
      const int end = (int)min((int64_t)__shfl(off + cnt, nw - 1), a.e_cap);  // no slots past the capacity
      float P[G_COUNT];
#pragma unroll
      for (int f = 0; f < G_COUNT; ++f) P[f] = 0.f;
      for (int w0 = base; w0 < end; w0 += 64) {
        const int e = w0 + lane;
        float r[G_COUNT];
        if (e < end) {
          entry_total(a.partials, a.used, e, r);
        } else {
#pragma unroll
          for (int f = 0; f < G_COUNT; ++f) r[f] = 0.f;
        }
#pragma unroll
        for (int f = 0; f < G_COUNT; ++f) rec[lane * kRecRow + f] = r[f];
        __builtin_amdgcn_wave_barrier();
        const int lo = max(off, w0), hi = min(min(off + cnt, w0 + 64), end);
        for (int j = lo; j < hi; ++j) {
          const float* t = rec + (j - w0) * kRecRow;
#pragma unroll
          for (int f = 0; f < G_COUNT; ++f) P[f] += t[f];
        }
        __builtin_amdgcn_wave_barrier();
      }
      if (cnt == 0) continue;
      const CamConst& c = cams.c[ci];
      gw += P[G_W];
      // emission colour
      float basis[16];
      bool live[3] = {true, true, true};
      if (DEG < 0) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) gcol[ch] += P[G_CR + ch];
      } else {
        float dx = mean[0] - c.o[0], dy = mean[1] - c.o[1], dz = mean[2] - c.o[2];
        float inv = rsqrtf(dx * dx + dy * dy + dz * dz);
        sh_basis(dx * inv, dy * inv, dz * inv, DEG, basis);
        const float* f = row;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
          float val = 0.5f;
#pragma unroll
          for (int k = 0; k < nsh; ++k) val += basis[k] * f[3 * k + ch];
          live[ch] = val > 0.f;
          if (live[ch]) {
#pragma unroll
            for (int k = 0; k < nsh; ++k) gcol[3 * k + ch] += P[G_CR + ch] * basis[k];
          }
        }
      }
      // coefficients -> (mean, scale, quat) in one reverse sweep
      coefs_adjoint(mean, scale, quat, c, P, gp);
      if (DEG >= 0) {
        // the SH view direction d = normalize(mean - origin) moves with the
        // mean: grad_d of S(d) = sum_k c_k Y_k(d), c_k the colour adjoints
        // contracted with the coefficients, projected off d and over |v|
        float dx = mean[0] - c.o[0], dy = mean[1] - c.o[1], dz = mean[2] - c.o[2];
        const float inv = rsqrtf(dx * dx + dy * dy + dz * dz);
        dx *= inv; dy *= inv; dz *= inv;
        float ck[16];
        const float* f = row;
#pragma unroll
        for (int k = 0; k < nsh; ++k) {
          float s = 0.f;
#pragma unroll
          for (int ch = 0; ch < 3; ++ch)
            if (live[ch]) s += P[G_CR + ch] * f[3 * k + ch];
          ck[k] = s;
        }
        float gd[3];
#pragma unroll 1
        for (int ax = 0; ax < 3; ++ax) {
          Dual bd[16];
          sh_basis(Dual(dx, ax == 0 ? 1.f : 0.f), Dual(dy, ax == 1 ? 1.f : 0.f), Dual(dz, ax == 2 ? 1.f : 0.f),
                   DEG, bd);
          float s = 0.f;
#pragma unroll
          for (int k = 0; k < nsh; ++k) s += ck[k] * bd[k].d;
          gd[ax] = s;
        }
        const float dd = gd[0] * dx + gd[1] * dy + gd[2] * dz;
        gp[0] += (gd[0] - dd * dx) * inv;
        gp[1] += (gd[1] - dd * dy) * inv;
        gp[2] += (gd[2] - dd * dz) * inv;
      }
    }
    if (valid) {
      a.g_means[3 * g] = gp[0]; a.g_means[3 * g + 1] = gp[1]; a.g_means[3 * g + 2] = gp[2];
      a.g_scales[3 * g] = gp[3]; a.g_scales[3 * g + 1] = gp[4]; a.g_scales[3 * g + 2] = gp[5];
      a.g_quats[4 * g] = gp[6]; a.g_quats[4 * g + 1] = gp[7]; a.g_quats[4 * g + 2] = gp[8];
      a.g_quats[4 * g + 3] = gp[9];
      a.g_dens[g] = gw;
#pragma unroll
      for (int k = 0; k < kPer; ++k) row[k] = gcol[k];  // this thread's row only
    }
  }
  __syncthreads();
  unstage_rows<kPer, kRow, 128>(a.g_colors + (size_t)g0 * kPer, shc, nblk);
}

hipError_t launch_grad_finalize(const GradArgs& a, const CamSet& cams, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  dim3 grid((a.n + 127) / 128), block(128);
  switch (a.sh_degree) {
    case -1: hipLaunchKernelGGL(k_grad_finalize<-1>, grid, block, 0, s, a, cams); break;
    case 0: hipLaunchKernelGGL(k_grad_finalize<0>, grid, block, 0, s, a, cams); break;
    case 1: hipLaunchKernelGGL(k_grad_finalize<1>, grid, block, 0, s, a, cams); break;
    case 2: hipLaunchKernelGGL(k_grad_finalize<2>, grid, block, 0, s, a, cams); break;
    case 3: hipLaunchKernelGGL(k_grad_finalize<3>, grid, block, 0, s, a, cams); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mb
