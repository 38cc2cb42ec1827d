// Host-side launch wrappers of the rendering kernels (one translation unit
// each); all enqueue on the given stream and return hipError_t.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace mb {

struct PrepArgs {
  const float *means, *scales, *quats, *dens, *colors;
  int n, sh_degree, tiles_x, tiles_y;
  double conf_term; // log(-log(1 - c) / sqrt(2 pi))
  int full_coverage;
  float4* rec;      // [C*n*6] render records
  double2* rectd;   // [C*n*3] exact rectangles: centre, major axis, halves
  int4* tbox;       // [C*n] tile box (tx0, ty0, tx1, ty1)
  int* counts;      // [C*n] overlapped tiles
  double* proxy_out; // optional [n*8] (camera 0)
};

hipError_t launch_preprocess(const PrepArgs& a, const CamSet& cams, hipStream_t s);

struct EmitArgs {
  const float4* rec;
  const int4* tbox;
  const int* offsets;  // [C*n] exclusive scan of counts
  const int* counts;   // [C*n] tiles counted by the preprocess kernel
  int n, n_cams, tiles_x, tiles_y, full_coverage;
  uint32_t* keys;      // [E] tile key cam * T + tile (the sort's values are the entry indices)
  int* entry_rec;      // [E] record index cam * n + g
  int2* ranges;        // [n_keys] cleared to (0, 0) when not null
  int n_keys;
  int64_t cap;         // entries at or beyond cap are not written (workspace capacity)
};
hipError_t launch_emit(const EmitArgs& a, hipStream_t s);

// D-SSIM loss (loss.hip).
struct SsimArgs {
  const float *image, *target;  // [C,H,W,3]
  int n_cams, w, h;
  float g[11];                  // normalised Gaussian window, sigma 1.5
  float* coef;                  // [C,H,W,3,3] dS/d(mu_x, E[x^2], E[xy]); null: loss only
  float* partials;              // [blocks]
  float* loss;                  // device scalar, 1 - mean SSIM
  float* grad;                  // [C,H,W,3] accumulated with grad_scale d loss / d image, or null
  float grad_scale;
};
hipError_t launch_dssim(const SsimArgs& a, hipStream_t s);
int l1_partials();
hipError_t launch_l1(const float* x, const float* y, int64_t n, float grad_scale, float* loss, float* grad,
                     double* partials, hipStream_t s);
int dssim_blocks(int n_cams, int w, int h);

// Adaptive density control (adc.hip).
enum AdcAction { kAdcPrune = 0, kAdcKeep = 1, kAdcClone = 2, kAdcSplit = 3 };
constexpr float kSplitGamma = 0.6385502815246582f;  // scale factor of the split axis (App. E)
constexpr float kSplitDelta = 0.6128153090966912f;  // offset of the split means, in units of that scale
struct AdcParams {
  float min_opacity, grad_threshold, split_scale;
};
struct AdcApplyArgs {
  int n, color_stride;
  const float *means, *scales, *quats, *dens, *colors;
  const int *action, *offsets;
  float *out_means, *out_scales, *out_quats, *out_dens, *out_colors;
};
hipError_t launch_vi_opacity(int n, const float* scales, const float* dens, float* o, hipStream_t s);
hipError_t launch_density_from_opacity(int n, const float* o, const float* scales, float* w, hipStream_t s);
hipError_t launch_adc_accumulate(int n, const float* g, float* acc, int* cnt, hipStream_t s);
hipError_t launch_adc_plan(int n, const float* scales, const float* dens, const float* acc, const int* cnt,
                           const AdcParams& p, int* action, int* outs, int* offsets, int* scan_tmp, int* total,
                           hipStream_t s);
hipError_t launch_adc_apply(const AdcApplyArgs& a, hipStream_t s);

// exclusive scan of int32 counts (n items) into out (n items), total in *total.
// tmp must hold scan_tmp_ints(n) ints.
size_t scan_tmp_ints(int64_t n);
hipError_t launch_scan(const int* in, int* out, int64_t n, int* tmp, int* total, hipStream_t s);

// stable LSD radix sort of (keys, vals) on the low `bits` bits of keys.
// Buffers *_a hold the input and receive the output; *_b are scratch. The
// launch is sized for n items; with n_dev the count is min(*n_dev, n), read
// on the device. identity_vals: the input values are 0, 1, 2, ... and vals_a
// is not read.
size_t radix_tmp_ints(int64_t n);
hipError_t launch_radix_sort(uint32_t* keys_a, int* vals_a, uint32_t* keys_b, int* vals_b,
                             int64_t n, const int* n_dev, int bits, int* tmp, hipStream_t s,
                             bool identity_vals = false);

// after the sort: sorted_rec[i] = entry_rec[vals[i]], ranges[key] =
// [first, last+1) over the sorted keys (ranges zeroed first, here unless
// ranges_cleared: the emit kernel clears them when given them).
hipError_t launch_finish_lists(const uint32_t* keys, const int* vals, const int* entry_rec,
                               int64_t n, const int* n_dev, int* sorted_rec, int2* ranges,
                               int n_keys, bool ranges_cleared, hipStream_t s);

// block list of the render kernels (render_blocks(n_keys) entries): tiles
// longer than `split` entries first, as four quadrant blocks, then the rest,
// each group by decreasing (quantised) list length; tmp holds
// order_tmp_ints(n_keys) ints
size_t order_tmp_ints(int n_keys);
hipError_t launch_tile_order(const int2* ranges, int n_keys, int split, int* blocks, int* tmp, hipStream_t s);

struct RenderArgs {
  const float4* rec;
  const double2* rectd;  // [C*n*3] exact rectangles (the coverage test near an edge)
  const int* sorted_rec;
  const int2* ranges;
  const int* order;  // [render_blocks(n_keys)] block list (see launch_tile_order)
  uint64_t* masks;   // [E,4] coverage of list entry (sorted position) by the pixels of wave w
  float* image;   // [C,H,W,3]
  float* saved;   // [C,H,W,8]
  int tiles_x, tiles_y, n_cams, full_coverage;
  float kappa, beta, eps;
  float xq[8];    // standard-normal edge quantiles
  float eq[8];    // exp(-kappa^2 xq^2 / 2)
  float ecq[8];   // erfc(kappa xq / sqrt2)
  float* penalty; // [C,H,W] consistency penalty per pixel, or null
  double* pix_mom; // [kMaxMoments + 1][C*H*W] per-pixel moment sums, written by the forward pass
  long long n_pix; // C*H*W
  // surrogate query list (emit / consume variants)
  float* pixfeat;                 // [C,H,W,kPixFeat] per-pixel features, m0, basis, count
  long long* pix_qbase;           // [C,H,W] first query of the pixel, -1 if none
  unsigned long long* q_count;    // queries requested (may exceed q_cap)
  long long q_cap;
  float* q_z;                     // [q_cap] standardised query
  int* q_pix;                     // [q_cap] flat pixel index
  const float* q_f;               // [q_cap] surrogate output F
  const float* q_g;               // [q_cap][8] F and dF/d(inputs) (backward through the surrogate)
  // tabulated schedule: [C*H*W][tab_nodes] reconstruction at the nodes
  float* tab;
  int tab_nodes;
  // training-sample harvest (harvest variant)
  float* harvest;                 // [harvest_cap, kHarvestStride]
  int* harvest_count;
  int harvest_cap;
  float harvest_rate;
  uint32_t seed;
};
// kModeTrig: the plain path with the trigonometric moments of Eqs. 13-14;
// kModeTabPlain / kModeTabSur: passes 0-1 and the per-pixel record of the
// tabulated schedule, with the table of the moment bounds (TabPlain) or the
// surrogate's inputs (TabSur); k_render_consume_tab completes the frame
enum RenderMode { kModePlain = 0, kModeHarvest = 1, kModeEmit = 2, kModeTrig = 3, kModeTabPlain = 4,
                  kModeTabSur = 5 };
hipError_t launch_render_forward(const RenderArgs& a, const CamSet& cams, int n_moments,
                                 int n_intervals, hipStream_t s, int mode = kModePlain);
hipError_t launch_render_consume(const RenderArgs& a, const CamSet& cams, int n_intervals, hipStream_t s);
hipError_t launch_render_consume_tab(const RenderArgs& a, const CamSet& cams, int n_intervals, hipStream_t s);

hipError_t launch_render_backward(const RenderArgs& r, const float* saved, const float* grad_image,
                                  const float* grad_penalty, const int* sorted_k, float* partials,
                                  uint8_t* used, const CamSet& cams, int n_moments, int n_intervals,
                                  hipStream_t s, int mode = 0);

struct GradArgs {
  const float *means, *scales, *quats, *dens, *colors;
  int n, sh_degree;
  const int* counts;     // [C*n]
  const int* offsets;    // [C*n]
  int64_t e_cap;         // entries with an index at or beyond e_cap have no slots
  const float* partials; // [E,4,kGradStride]
  const uint8_t* used;   // [E,4]: slot (entry, wave) holds data; its sum is zero otherwise
  float *g_means, *g_scales, *g_quats, *g_dens, *g_colors;
};
hipError_t launch_grad_finalize(const GradArgs& a, const CamSet& cams, hipStream_t s);

// learned surrogate (mlp.hip)
int mlp_param_count();
size_t mlp_packed_bytes();
size_t mlp_workspace_bytes(int64_t n);
hipError_t launch_mlp_pack(const float* theta, void* packed, hipStream_t s);
hipError_t launch_mlp_forward(const void* packed, const float* x, int64_t n, float* f, hipStream_t s);
// surrogate inputs gathered from the render's query list: features of pixel
// q_pix[i] (of n_pix) and query q_z[i] for i < min(*q_count, q_cap)
hipError_t launch_mlp_forward_gather(const void* packed, const float* pixfeat, int64_t n_pix, const int* q_pix,
                                     const float* q_z, const unsigned long long* q_count, int64_t q_cap, float* f,
                                     hipStream_t s);
// the surrogate at the n_nodes nodes of every pixel's table: tab[p][g] = F(features of p, z_g)
hipError_t launch_mlp_table(const void* packed, const float* pixfeat, int64_t n_pix, int n_nodes, float* tab,
                            hipStream_t s);
// F and dF/dinputs [q][8] for the render's query list (backward through the surrogate)
hipError_t launch_mlp_input_grad_gather(const void* packed, const float* pixfeat, int64_t n_pix, const int* q_pix,
                                        const float* q_z, const unsigned long long* q_count, int64_t q_cap,
                                        float* out_g, hipStream_t s);
hipError_t launch_mlp_loss_grad(const void* packed, const float* x, const float* t, int64_t n, float* grad,
                                float* loss, float* ws, hipStream_t s);
hipError_t launch_adam(float* th, float* m, float* v, const float* g, int64_t count, int step, float lr, float b1,
                       float b2, float eps, hipStream_t s);

}  // namespace mb
