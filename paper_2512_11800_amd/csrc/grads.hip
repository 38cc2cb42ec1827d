// Per-Gaussian end of the backward pass: sum the per-(list entry, wave) slots
// of the Gradient stage over every tile and camera the Gaussian was listed
// in (its entries are contiguous), then chain the record-coefficient
// gradients to mean, scale and rotation. The chain rule runs in forward mode
// through the same templated coefficient code the preprocess uses, one
// tangent per parameter, so there is a single definition of the geometry.
#include "kernels.h"

namespace mb {

// The block's colour coefficients are staged through LDS (one padded row per
// Gaussian) so their loads and the colour-gradient stores are coalesced.
template <int DEG>
__global__ __launch_bounds__(128) void k_grad_finalize(GradArgs a, CamSet cams) {
  constexpr int nsh = DEG < 0 ? 1 : (DEG + 1) * (DEG + 1);
  constexpr int kPer = 3 * nsh;
  constexpr int kRow = kPer | 1;
  __shared__ float shc[128 * kRow];
  const int g0 = blockIdx.x * blockDim.x;
  const int nblk = min(128, a.n - g0);
  for (int i = threadIdx.x; i < nblk * kPer; i += 128)
    shc[(i / kPer) * kRow + i % kPer] = a.colors[(size_t)g0 * kPer + i];
  __syncthreads();
  float* row = shc + threadIdx.x * kRow;
  int g = g0 + threadIdx.x;
  if (g < a.n) {
    float mean[3] = {a.means[3 * g], a.means[3 * g + 1], a.means[3 * g + 2]};
    float scale[3] = {a.scales[3 * g], a.scales[3 * g + 1], a.scales[3 * g + 2]};
    float quat[4] = {a.quats[4 * g], a.quats[4 * g + 1], a.quats[4 * g + 2], a.quats[4 * g + 3]};
    float gp[10];
#pragma unroll
    for (int p = 0; p < 10; ++p) gp[p] = 0.f;
    float gw = 0.f;
    float gcol[3 * nsh];
#pragma unroll
    for (int k = 0; k < 3 * nsh; ++k) gcol[k] = 0.f;

    for (int ci = 0; ci < cams.n_cams; ++ci) {
      size_t idx = (size_t)ci * a.n + g;
      int cnt = a.counts[idx];
      if (cnt == 0) continue;
      const CamConst& c = cams.c[ci];
      int off = a.offsets[idx];
      float P[G_COUNT];
#pragma unroll
      for (int f = 0; f < G_COUNT; ++f) P[f] = 0.f;
      for (int e = 0; e < cnt; ++e) {
        const float4* sl = reinterpret_cast<const float4*>(a.partials + (size_t)(off + e) * 4 * kGradStride);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const float4* s = sl + w * (kGradStride / 4);
          float4 v0 = s[0], v1 = s[1], v2 = s[2], v3 = s[3], v4 = s[4];
          P[0] += v0.x; P[1] += v0.y; P[2] += v0.z; P[3] += v0.w;
          P[4] += v1.x; P[5] += v1.y; P[6] += v1.z; P[7] += v1.w;
          P[8] += v2.x; P[9] += v2.y; P[10] += v2.z; P[11] += v2.w;
          P[12] += v3.x; P[13] += v3.y; P[14] += v3.z; P[15] += v3.w;
          P[16] += v4.x; P[17] += v4.y;
        }
      }
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
      // coefficients -> (mean, scale, quat), one tangent at a time
#pragma unroll 1
      for (int p = 0; p < 10; ++p) {
        Dual md[3], sd[3], qd[4];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          md[k] = Dual(mean[k], p == k ? 1.f : 0.f);
          sd[k] = Dual(scale[k], p == 3 + k ? 1.f : 0.f);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) qd[k] = Dual(quat[k], p == 6 + k ? 1.f : 0.f);
        Coefs<Dual> cf;
        compute_coefs(md, sd, qd, c, cf);
        float d = P[G_D0] * cf.D0.d + P[G_D1X] * cf.D1x.d + P[G_D1Y] * cf.D1y.d + P[G_D2XX] * cf.D2xx.d +
                  P[G_D2XY] * cf.D2xy.d + P[G_D2YY] * cf.D2yy.d + P[G_E0] * cf.E0.d + P[G_EX] * cf.Ex.d +
                  P[G_EY] * cf.Ey.d + P[G_XXX] * cf.Xxx.d + P[G_XXY] * cf.Xxy.d + P[G_XYY] * cf.Xyy.d +
                  P[G_P0X] * cf.p0x.d + P[G_P0Y] * cf.p0y.d;
        if (DEG >= 0 && p < 3) {
          // the SH view direction normalize(mean - origin) moves with the mean
          Dual ddx = md[0] - Dual(c.o[0]), ddy = md[1] - Dual(c.o[1]), ddz = md[2] - Dual(c.o[2]);
          Dual nrm = dsqrt(ddx * ddx + ddy * ddy + ddz * ddz);
          Dual bd[16];
          sh_basis(ddx / nrm, ddy / nrm, ddz / nrm, DEG, bd);
          const float* f = row;
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) {
            if (!live[ch]) continue;
            float dv = 0.f;
#pragma unroll
            for (int k = 0; k < nsh; ++k) dv += bd[k].d * f[3 * k + ch];
            d += P[G_CR + ch] * dv;
          }
        }
        gp[p] += d;
      }
    }
    a.g_means[3 * g] = gp[0]; a.g_means[3 * g + 1] = gp[1]; a.g_means[3 * g + 2] = gp[2];
    a.g_scales[3 * g] = gp[3]; a.g_scales[3 * g + 1] = gp[4]; a.g_scales[3 * g + 2] = gp[5];
    a.g_quats[4 * g] = gp[6]; a.g_quats[4 * g + 1] = gp[7]; a.g_quats[4 * g + 2] = gp[8]; a.g_quats[4 * g + 3] = gp[9];
    a.g_dens[g] = gw;
#pragma unroll
    for (int k = 0; k < kPer; ++k) row[k] = gcol[k];  // this thread's row only
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nblk * kPer; i += 128)
    a.g_colors[(size_t)g0 * kPer + i] = shc[(i / kPer) * kRow + i % kPer];
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
