// Adaptive density control of the density-based medium (the training
// paragraph of Sec. 4 and App. E): the view-independent opacity used for
// pruning and for initial peak densities, accumulation of the absolute mean
// gradient that decides densification, and one densify/prune step (clone at
// half density, deterministic split along the longest axis). One thread per
// particle throughout; the output layout of a step comes from an exclusive
// scan of the per-particle output counts.
#include "kernels.h"

namespace mb {

constexpr float kSqrt2Pi = 2.5066282746310002f;

__global__ __launch_bounds__(256) void k_vi_opacity(int n, const float* scales, const float* dens, float* o) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float s = fminf(fminf(scales[3 * i], scales[3 * i + 1]), scales[3 * i + 2]);
  o[i] = -expm1f(-kSqrt2Pi * dens[i] * s);
}

__global__ __launch_bounds__(256) void k_density_from_opacity(int n, const float* o, const float* scales, float* w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float s = (scales[3 * i] + scales[3 * i + 1] + scales[3 * i + 2]) * (1.f / 3.f);
  w[i] = -log1pf(-o[i]) / (kSqrt2Pi * s);
}

__global__ __launch_bounds__(256) void k_adc_accumulate(int n, const float* g, float* acc, int* cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gx = g[3 * i], gy = g[3 * i + 1], gz = g[3 * i + 2];
  acc[3 * i] += fabsf(gx);
  acc[3 * i + 1] += fabsf(gy);
  acc[3 * i + 2] += fabsf(gz);
  cnt[i] += (gx != 0.f || gy != 0.f || gz != 0.f) ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_adc_plan(int n, const float* scales, const float* dens, const float* acc,
                                                  const int* cnt, AdcParams p, int* action, int* outs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float s0 = scales[3 * i], s1 = scales[3 * i + 1], s2 = scales[3 * i + 2];
  const float o = -expm1f(-kSqrt2Pi * dens[i] * fminf(fminf(s0, s1), s2));
  const float ax = acc[3 * i], ay = acc[3 * i + 1], az = acc[3 * i + 2];
  const int c = cnt[i];
  const float g = sqrtf(ax * ax + ay * ay + az * az) / (float)max(c, 1);
  int a = kAdcKeep;
  if (o < p.min_opacity)
    a = kAdcPrune;
  else if (c > 0 && g > p.grad_threshold)
    a = fmaxf(fmaxf(s0, s1), s2) > p.split_scale ? kAdcSplit : kAdcClone;
  action[i] = a;
  outs[i] = a == kAdcPrune ? 0 : (a == kAdcKeep ? 1 : 2);
}

__global__ __launch_bounds__(256) void k_adc_apply(AdcApplyArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int act = a.action[i];
  if (act == kAdcPrune) return;
  const int o = a.offsets[i];
  const float m[3] = {a.means[3 * i], a.means[3 * i + 1], a.means[3 * i + 2]};
  const float s[3] = {a.scales[3 * i], a.scales[3 * i + 1], a.scales[3 * i + 2]};
  const float q[4] = {a.quats[4 * i], a.quats[4 * i + 1], a.quats[4 * i + 2], a.quats[4 * i + 3]};
  const float w = a.dens[i];
  const int copies = act == kAdcKeep ? 1 : 2;
  float off[3] = {0.f, 0.f, 0.f};
  float sn[3] = {s[0], s[1], s[2]};
  float wn = act == kAdcClone ? 0.5f * w : w;  // the two copies together are the original density
  if (act == kAdcSplit) {
    // the axis of the largest scale: that column of the rotation matrix
    const int k = (s[0] >= s[1] && s[0] >= s[2]) ? 0 : (s[1] >= s[2] ? 1 : 2);
    const float qn = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const float qw = q[0] / qn, qx = q[1] / qn, qy = q[2] / qn, qz = q[3] / qn;
    float col[3];
    if (k == 0) {
      col[0] = 1.f - 2.f * (qy * qy + qz * qz); col[1] = 2.f * (qx * qy + qw * qz); col[2] = 2.f * (qx * qz - qw * qy);
    } else if (k == 1) {
      col[0] = 2.f * (qx * qy - qw * qz); col[1] = 1.f - 2.f * (qx * qx + qz * qz); col[2] = 2.f * (qy * qz + qw * qx);
    } else {
      col[0] = 2.f * (qx * qz + qw * qy); col[1] = 2.f * (qy * qz - qw * qx); col[2] = 1.f - 2.f * (qx * qx + qy * qy);
    }
    const float d = kSplitDelta * s[k];
#pragma unroll
    for (int c = 0; c < 3; ++c) off[c] = d * col[c];
    sn[k] = kSplitGamma * s[k];
  }
  for (int r = 0; r < copies; ++r) {
    const int t = o + r;
    const float sign = act == kAdcSplit ? (r == 0 ? -1.f : 1.f) : 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      a.out_means[3 * t + c] = m[c] + sign * off[c];
      a.out_scales[3 * t + c] = sn[c];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) a.out_quats[4 * t + c] = q[c];
    a.out_dens[t] = wn;
    for (int c = 0; c < a.color_stride; ++c)
      a.out_colors[(size_t)t * a.color_stride + c] = a.colors[(size_t)i * a.color_stride + c];
  }
}

static dim3 grid_of(int n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t launch_vi_opacity(int n, const float* scales, const float* dens, float* o, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_vi_opacity, grid_of(n), dim3(256), 0, s, n, scales, dens, o);
  return hipGetLastError();
}

hipError_t launch_density_from_opacity(int n, const float* o, const float* scales, float* w, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_density_from_opacity, grid_of(n), dim3(256), 0, s, n, o, scales, w);
  return hipGetLastError();
}

hipError_t launch_adc_accumulate(int n, const float* g, float* acc, int* cnt, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adc_accumulate, grid_of(n), dim3(256), 0, s, n, g, acc, cnt);
  return hipGetLastError();
}

hipError_t launch_adc_plan(int n, const float* scales, const float* dens, const float* acc, const int* cnt,
                           const AdcParams& p, int* action, int* outs, int* offsets, int* scan_tmp, int* total,
                           hipStream_t s) {
  if (n > 0) {
    hipLaunchKernelGGL(k_adc_plan, grid_of(n), dim3(256), 0, s, n, scales, dens, acc, cnt, p, action, outs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return launch_scan(outs, offsets, n, scan_tmp, total, s);
}

hipError_t launch_adc_apply(const AdcApplyArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adc_apply, grid_of(a.n), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace mb
