// Per (camera, Gaussian) setup: frustum culling with the bounding sphere
// (Sec. 3.3), the confidence-interval screen proxy (Eqs. 16-21, App. D), the
// ray-space coefficients of the render record, the emission colour, and the
// 16x16 tiles the proxy rectangle overlaps; then emission of the tile lists.
#include "kernels.h"

namespace mb {

// Oriented rectangle of the level set omega(d) = C (App. D), in double.
// With delta = 2 (log w - log C), the pixel offset satisfies omega >= C iff
// X(delta) <= delta D(delta) (the paper's conic p^T W p >= 0 with
// W = m m^T - kappa M, kappa = mean^T A mean - delta, rewritten around the
// projected mean): Q = X2 - delta D2, centre Q^-1 (delta D1), and
// Sigma_2d = (delta D0 + delta D1 . centre) Q^-1. The first axis is the
// ellipse's major axis at theta = atan2(2 s_xy, s_xx - s_yy) / 2 of Sigma_2d,
// which is proportional to [[q_yy, -q_xy], [-q_xy, q_xx]]; a circle takes
// theta = 0. Every decision of the render (cull, rectangle, pixel coverage)
// is taken in double, so it is fixed by the float32 inputs alone.
struct RectD {
  double rcx, rcy, e1x, e1y, h1, h2;  // centre offset from the projected mean, major axis, halves
};

__device__ __forceinline__ bool proxy_rect(const Coefs<double>& cf, double w, double conf_term, RectD& r) {
  double quad = cf.mug[0] * cf.mug[0] + cf.mug[1] * cf.mug[1] + cf.mug[2] * cf.mug[2];
  double mc2 = cf.muc[0] * cf.muc[0] + cf.muc[1] * cf.muc[1] + cf.muc[2] * cf.muc[2];
  if (!(w > 0.0)) return false;
  double log_c = conf_term + 0.5 * log(quad / mc2);
  double delta = 2.0 * (log(w) - log_c);
  // real ellipse: peak opacity above c (delta > 0) and the camera outside the
  // confidence region (kappa = quad - delta > 0)
  if (!(delta > 0.0) || !(delta < quad)) return false;
  double qxx = cf.Xxx - delta * cf.D2xx;
  double qxy = cf.Xxy - delta * cf.D2xy;
  double qyy = cf.Xyy - delta * cf.D2yy;
  double det = qxx * qyy - qxy * qxy;
  if (!(qxx > 0.0) || !(qyy > 0.0) || !(det > 0.0)) return false;
  double bx = delta * cf.D1x, by = delta * cf.D1y;
  double cx = (qyy * bx - qxy * by) / det;
  double cy = (qxx * by - qxy * bx) / det;
  double r2 = delta * cf.D0 + bx * cx + by * cy;
  if (!(r2 > 0.0)) return false;
  double mid = 0.5 * (qxx + qyy);
  double rad = sqrt(0.25 * (qxx - qyy) * (qxx - qyy) + qxy * qxy);
  double ql = mid + rad;  // larger eigenvalue of Q: the minor axis of the ellipse
  double qs = det / ql;
  double th = 0.5 * atan2(-qxy, 0.5 * (qyy - qxx));
  r.rcx = cx; r.rcy = cy;
  r.e1x = cos(th); r.e1y = sin(th);
  r.h1 = sqrt(r2 / qs);
  r.h2 = sqrt(r2 / ql);
  return isfinite(r.h1) && isfinite(r.h2) && isfinite(cx) && isfinite(cy);
}

// float copy of the rectangle for the binning and the render record
struct Rect {
  float rcx, rcy, e1x, e1y, h1, h2;
};

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
  const double mean[3] = {a.means[3 * g], a.means[3 * g + 1], a.means[3 * g + 2]};
  const double scale[3] = {a.scales[3 * g], a.scales[3 * g + 1], a.scales[3 * g + 2]};
  const double quat[4] = {a.quats[4 * g], a.quats[4 * g + 1], a.quats[4 * g + 2], a.quats[4 * g + 3]};
  const float w = a.dens[g];

  Coefs<double> cf;
  compute_coefs(mean, scale, quat, c, cf);

  // --- culling: bounding sphere r = max diag S against the frustum --------
  const double rad = fmax(scale[0], fmax(scale[1], scale[2]));
  const double z = cf.muc[2], tn = c.tn;
  bool keep = (z > tn) && (z + rad >= tn);
  {
    const double fx = c.fx, fy = c.fy, cx = c.cx, cy = c.cy;
    const double nv[4][3] = {{fx, 0.0, cx}, {-fx, 0.0, (double)c.width - cx},
                             {0.0, fy, cy}, {0.0, -fy, (double)c.height - cy}};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double len = sqrt(nv[k][0] * nv[k][0] + nv[k][1] * nv[k][1] + nv[k][2] * nv[k][2]);
      const double d = (nv[k][0] * cf.muc[0] + nv[k][1] * cf.muc[1] + nv[k][2] * cf.muc[2]) / len + rad;
      keep = keep && (d >= 0.0);
    }
  }
  // the render record keeps the projected mean in float; the rectangle's
  // centre is stored as an offset from that float position
  const float p0x = (float)cf.p0x, p0y = (float)cf.p0y;
  RectD rd{0.0, 0.0, 1.0, 0.0, 0.0, 0.0};
  if (a.full_coverage) {
    keep = z > 0.0;
    rd.rcx = 0.5 * c.width - (double)p0x;
    rd.rcy = 0.5 * c.height - (double)p0y;
    rd.e1x = 1.0; rd.e1y = 0.0;
    rd.h1 = 0.5 * c.width + 1.0;
    rd.h2 = 0.5 * c.height + 1.0;
  } else {
    keep = keep && proxy_rect(cf, (double)w, a.conf_term, rd);
    rd.rcx += cf.p0x - (double)p0x;
    rd.rcy += cf.p0y - (double)p0y;
  }
  const Rect r{(float)rd.rcx, (float)rd.rcy, (float)rd.e1x, (float)rd.e1y, (float)rd.h1, (float)rd.h2};
  float mx = p0x + r.rcx, my = p0y + r.rcy;
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
    double* po = a.proxy_out + 8 * (size_t)g;
    po[0] = (double)p0x + rd.rcx; po[1] = (double)p0y + rd.rcy;
    po[2] = rd.e1x; po[3] = rd.e1y; po[4] = rd.h1; po[5] = rd.h2;
    po[6] = keep ? 1.0 : 0.0; po[7] = 0.0;
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
    float dx = a.means[3 * g] - c.o[0], dy = a.means[3 * g + 1] - c.o[1], dz = a.means[3 * g + 2] - c.o[2];
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
  float4* out = a.rec + idx * kRecStride;
  out[0] = make_float4(p0x, p0y, r.rcx, r.rcy);
  out[1] = make_float4(r.e1x, r.e1y, r.h1, r.h2);
  out[2] = make_float4((float)cf.D0, (float)cf.D1x, (float)cf.D1y, (float)cf.D2xx);
  out[3] = make_float4((float)cf.D2xy, (float)cf.D2yy, (float)cf.E0, (float)cf.Ex);
  out[4] = make_float4((float)cf.Ey, (float)cf.Xxx, (float)cf.Xxy, (float)cf.Xyy);
  out[5] = make_float4(w, rgb[0], rgb[1], rgb[2]);
  // the exact rectangle: absolute centre, major axis, halves
  double2* od = a.rectd + idx * 3;
  od[0] = make_double2((double)p0x + rd.rcx, (double)p0y + rd.rcy);
  od[1] = make_double2(rd.e1x, rd.e1y);
  od[2] = make_double2(rd.h1, rd.h2);
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
  const float4* rp = a.rec + idx * kRecStride;
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
