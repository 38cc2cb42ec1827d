// Per (camera, Gaussian) setup: frustum culling with the bounding sphere
// (Sec. 3.3), the confidence-interval screen proxy (Eqs. 16-21, App. D), the
// ray-space coefficients of the render record, the emission colour, and the
// 16x16 tiles the proxy rectangle overlaps; then emission of the tile lists.
#include "kernels.h"

namespace mb {

// Oriented rectangle of the level set omega(d) = C (App. D).
// With delta = 2 (log w - log C), the pixel offset satisfies omega >= C iff
// X(delta) <= delta D(delta) (the paper's conic p^T W p >= 0 with
// W = m m^T - kappa M, kappa = mean^T A mean - delta, rewritten around the
// projected mean): Q = X2 - delta D2, centre Q^-1 (delta D1), and
// Sigma_2d = (delta D0 + delta D1 . centre) Q^-1, whose eigenpairs span the box.
struct Rect {
  float rcx, rcy, e1x, e1y, h1, h2;
};

__device__ __forceinline__ bool proxy_rect(const Coefs<float>& cf, float w, float conf_term, Rect& r) {
  float quad = cf.mug[0] * cf.mug[0] + cf.mug[1] * cf.mug[1] + cf.mug[2] * cf.mug[2];
  float mc2 = cf.muc[0] * cf.muc[0] + cf.muc[1] * cf.muc[1] + cf.muc[2] * cf.muc[2];
  if (!(w > 0.f)) return false;
  float log_c = conf_term + 0.5f * logf(quad / mc2);
  float delta = 2.f * (logf(w) - log_c);
  // real ellipse: peak opacity above c (delta > 0) and the camera outside the
  // confidence region (kappa = quad - delta > 0)
  if (!(delta > 0.f) || !(delta < quad)) return false;
  float qxx = cf.Xxx - delta * cf.D2xx;
  float qxy = cf.Xxy - delta * cf.D2xy;
  float qyy = cf.Xyy - delta * cf.D2yy;
  float det = qxx * qyy - qxy * qxy;
  if (!(qxx > 0.f) || !(qyy > 0.f) || !(det > 0.f)) return false;
  float bx = delta * cf.D1x, by = delta * cf.D1y;
  float cx = (qyy * bx - qxy * by) / det;
  float cy = (qxx * by - qxy * bx) / det;
  float r2 = delta * cf.D0 + bx * cx + by * cy;
  if (!(r2 > 0.f)) return false;
  float mid = 0.5f * (qxx + qyy);
  float rad = sqrtf(0.25f * (qxx - qyy) * (qxx - qyy) + qxy * qxy);
  float ql = mid + rad;
  float qs = det / ql;
  // eigenvector of the larger eigenvalue of Q (shorter axis of the ellipse)
  float ax = qxy, ay = ql - qxx;
  float bx2 = ql - qyy, by2 = qxy;
  float na = ax * ax + ay * ay, nb = bx2 * bx2 + by2 * by2;
  float ex, ey;
  if (na >= nb) { ex = ax; ey = ay; } else { ex = bx2; ey = by2; na = nb; }
  if (na > 0.f) {
    float inv = rsqrtf(na);
    ex *= inv; ey *= inv;
  } else {
    ex = 1.f; ey = 0.f;
  }
  r.rcx = cx; r.rcy = cy; r.e1x = ex; r.e1y = ey;
  r.h1 = sqrtf(r2 / ql);
  r.h2 = sqrtf(r2 / qs);
  return isfinite(r.h1) && isfinite(r.h2) && isfinite(cx) && isfinite(cy);
}

// Does the rectangle (centre m, axes e1/e2, halves h) reach a pixel centre
// of tile (tx, ty)? Separating-axis test of the rectangle against the box of
// the tile's pixel centres, slightly enlarged so no covered pixel is missed.
__device__ __forceinline__ bool tile_overlaps(float mx, float my, const Rect& r, int tx, int ty) {
  // evaluated identically by the counting and the emitting kernel
#pragma clang fp contract(off)
  const float margin = 1e-2f;
  float dx = (float)(tx * kTile) + 8.f - mx;
  float dy = (float)(ty * kTile) + 8.f - my;
  float ext = 7.5f * (fabsf(r.e1x) + fabsf(r.e1y));
  float p1 = fabsf(dx * r.e1x + dy * r.e1y);
  float p2 = fabsf(-dx * r.e1y + dy * r.e1x);
  return p1 <= r.h1 + ext + margin && p2 <= r.h2 + ext + margin;
}

__device__ __forceinline__ bool tile_box(float mx, float my, const Rect& r, int width, int height,
                                         int tiles_x, int tiles_y, int4& box) {
#pragma clang fp contract(off)
  const float margin = 1e-2f;
  float ex = r.h1 * fabsf(r.e1x) + r.h2 * fabsf(r.e1y) + margin;
  float ey = r.h1 * fabsf(r.e1y) + r.h2 * fabsf(r.e1x) + margin;
  float xl = mx - ex - 0.5f, xh = mx + ex - 0.5f;
  float yl = my - ey - 0.5f, yh = my + ey - 0.5f;
  if (!(xh >= 0.f) || !(yh >= 0.f) || !(xl <= (float)(width - 1)) || !(yl <= (float)(height - 1)))
    return false;
  int x0 = (int)ceilf(fmaxf(xl, 0.f)), x1 = (int)floorf(fminf(xh, (float)(width - 1)));
  int y0 = (int)ceilf(fmaxf(yl, 0.f)), y1 = (int)floorf(fminf(yh, (float)(height - 1)));
  if (x0 > x1 || y0 > y1) return false;
  box = make_int4(x0 / kTile, y0 / kTile, min(x1 / kTile, tiles_x - 1), min(y1 / kTile, tiles_y - 1));
  return true;
}

// DEG: SH degree (-1 for plain RGB). The block's SH coefficients are first
// copied to LDS with coalesced loads (a Gaussian's 48 floats are contiguous,
// so per-thread reads would touch 64 cache lines per instruction), one padded
// row per Gaussian against bank conflicts.
template <int DEG>
__global__ __launch_bounds__(256) void k_preprocess(PrepArgs a, CamSet cams) {
  constexpr int kPer = DEG < 0 ? 3 : (DEG + 1) * (DEG + 1) * 3;
  constexpr int kRow = kPer | 1;
  __shared__ float shc[256 * kRow];
  {
    const int g0 = blockIdx.x * blockDim.x;
    stage_rows<kPer, kRow, 256>(shc, a.colors + (size_t)g0 * kPer, min(256, a.n - g0));
    __syncthreads();
  }
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  int ci = blockIdx.y;
  if (g >= a.n) return;
  const CamConst& c = cams.c[ci];
  size_t idx = (size_t)ci * a.n + g;
  float mean[3] = {a.means[3 * g], a.means[3 * g + 1], a.means[3 * g + 2]};
  float scale[3] = {a.scales[3 * g], a.scales[3 * g + 1], a.scales[3 * g + 2]};
  float quat[4] = {a.quats[4 * g], a.quats[4 * g + 1], a.quats[4 * g + 2], a.quats[4 * g + 3]};
  float w = a.dens[g];

  Coefs<float> cf;
  compute_coefs(mean, scale, quat, c, cf);

  // --- culling: bounding sphere r = max diag S against the frustum --------
  float rad = fmaxf(scale[0], fmaxf(scale[1], scale[2]));
  float z = cf.muc[2];
  bool keep = (z > c.tn) && (z + rad >= c.tn);
  {
    float nl[3] = {c.fx, 0.f, c.cx};
    float nr[3] = {-c.fx, 0.f, (float)c.width - c.cx};
    float nt[3] = {0.f, c.fy, c.cy};
    float nb[3] = {0.f, -c.fy, (float)c.height - c.cy};
    const float* ns[4] = {nl, nr, nt, nb};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float* nv = ns[k];
      float inv = rsqrtf(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
      float d = (nv[0] * cf.muc[0] + nv[1] * cf.muc[1] + nv[2] * cf.muc[2]) * inv + rad;
      keep = keep && (d >= 0.f);
    }
  }
  Rect r;
  if (a.full_coverage) {
    keep = z > 0.f;
    r.rcx = 0.5f * (float)c.width - cf.p0x;
    r.rcy = 0.5f * (float)c.height - cf.p0y;
    r.e1x = 1.f; r.e1y = 0.f;
    r.h1 = 0.5f * (float)c.width + 1.f;
    r.h2 = 0.5f * (float)c.height + 1.f;
  } else {
    keep = keep && proxy_rect(cf, w, a.conf_term, r);
  }
  float mx = cf.p0x + r.rcx, my = cf.p0y + r.rcy;
  int4 box = make_int4(0, 0, -1, -1);
  int count = 0;
  if (keep && tile_box(mx, my, r, c.width, c.height, a.tiles_x, a.tiles_y, box)) {
    for (int ty = box.y; ty <= box.w; ++ty)
      for (int tx = box.x; tx <= box.z; ++tx) count += tile_overlaps(mx, my, r, tx, ty) ? 1 : 0;
  } else {
    box = make_int4(0, 0, -1, -1);
    keep = false;
  }
  if (a.proxy_out != nullptr && ci == 0) {
    float* po = a.proxy_out + 8 * (size_t)g;
    po[0] = mx; po[1] = my; po[2] = r.e1x; po[3] = r.e1y; po[4] = r.h1; po[5] = r.h2;
    po[6] = keep ? 1.f : 0.f; po[7] = 0.f;
  }
  if (a.counts == nullptr) return;
  a.counts[idx] = count;
  a.tbox[idx] = box;
  if (count == 0) return;

  // --- emission colour: RGB or SH at the per-Gaussian view direction ------
  float rgb[3];
  const float* f = shc + threadIdx.x * kRow;
  if constexpr (DEG < 0) {
    rgb[0] = f[0]; rgb[1] = f[1]; rgb[2] = f[2];
  } else {
    constexpr int nb = (DEG + 1) * (DEG + 1);
    float dx = mean[0] - c.o[0], dy = mean[1] - c.o[1], dz = mean[2] - c.o[2];
    float inv = rsqrtf(dx * dx + dy * dy + dz * dz);
    float basis[16];
    sh_basis(dx * inv, dy * inv, dz * inv, DEG, basis);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      float v = 0.5f;
#pragma unroll
      for (int k = 0; k < nb; ++k) v += basis[k] * f[3 * k + ch];
      rgb[ch] = fmaxf(v, 0.f);
    }
  }
  float4* out = a.rec + idx * kRecF4;
  out[0] = make_float4(cf.p0x, cf.p0y, r.rcx, r.rcy);
  out[1] = make_float4(r.e1x, r.e1y, r.h1, r.h2);
  out[2] = make_float4(cf.D0, cf.D1x, cf.D1y, cf.D2xx);
  out[3] = make_float4(cf.D2xy, cf.D2yy, cf.E0, cf.Ex);
  out[4] = make_float4(cf.Ey, cf.Xxx, cf.Xxy, cf.Xyy);
  out[5] = make_float4(w, rgb[0], rgb[1], rgb[2]);
}

hipError_t launch_preprocess(const PrepArgs& a, const CamSet& cams, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  dim3 grid((a.n + 255) / 256, cams.n_cams);
  switch (a.sh_degree) {
    case -1: hipLaunchKernelGGL(k_preprocess<-1>, grid, dim3(256), 0, s, a, cams); break;
    case 0: hipLaunchKernelGGL(k_preprocess<0>, grid, dim3(256), 0, s, a, cams); break;
    case 1: hipLaunchKernelGGL(k_preprocess<1>, grid, dim3(256), 0, s, a, cams); break;
    case 2: hipLaunchKernelGGL(k_preprocess<2>, grid, dim3(256), 0, s, a, cams); break;
    case 3: hipLaunchKernelGGL(k_preprocess<3>, grid, dim3(256), 0, s, a, cams); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_emit(EmitArgs a) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  int ci = blockIdx.y;
  if (a.ranges) {  // empty per-tile ranges, filled in after the sort
    const int nt = gridDim.x * gridDim.y * blockDim.x;
    for (int t = (blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x; t < a.n_keys; t += nt)
      a.ranges[t] = make_int2(0, 0);
  }
  if (g >= a.n) return;
  size_t idx = (size_t)ci * a.n + g;
  int4 box = a.tbox[idx];
  if (box.x > box.z) return;
  const float4* rp = a.rec + idx * kRecF4;
  float4 r0 = rp[0], r1 = rp[1];
  Rect r{r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
  float mx = r0.x + r0.z, my = r0.y + r0.w;
  int off = a.offsets[idx];
  int count = a.counts[idx];
  uint32_t base_key = (uint32_t)ci * (uint32_t)(a.tiles_x * a.tiles_y);
  // entries past the workspace capacity are dropped (the caller compares the
  // count with its capacity and renders again)
  if (off >= a.cap) return;
  count = (int)min((int64_t)count, a.cap - off);
  int j = 0;
  for (int ty = box.y; ty <= box.w && j < count; ++ty)
    for (int tx = box.x; tx <= box.z && j < count; ++tx) {
      if (!tile_overlaps(mx, my, r, tx, ty)) continue;
      int e = off + j++;
      a.keys[e] = base_key + (uint32_t)(ty * a.tiles_x + tx);
      a.entry_rec[e] = (int)idx;
    }
  // never leave a counted slot unwritten; an extra list entry is harmless
  // because the render kernels test coverage per pixel
  for (; j < count; ++j) {
    int e = off + j;
    a.keys[e] = base_key + (uint32_t)(box.y * a.tiles_x + box.x);
    a.entry_rec[e] = (int)idx;
  }
}

hipError_t launch_emit(const EmitArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  dim3 grid((a.n + 255) / 256, a.n_cams);
  hipLaunchKernelGGL(k_emit, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace mb
