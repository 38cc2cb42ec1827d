/*
 * mb3dgs.h -- C ABI of the MI355X (gfx950) rendering path of moment-based
 * order-independent 3D Gaussian splatting (arXiv 2512.11800).
 *
 * The library renders a set of 3D Gaussians (mean, scale, rotation,
 * non-negative density weight, colour or SH coefficients; Sec. 3.1) from one
 * or more pinhole cameras. Per pixel it accumulates warped power moments of
 * the optical depth in closed form (Sec. 3.2, Eqs. 10-12), reconstructs the
 * optical depth from them with moment bounds (Sec. 3.2), integrates each
 * covering Gaussian with the piecewise-constant quadrature of Eq. 7 (App. B)
 * and rescales by the true opacity (Eq. 15). Gaussians are rasterised through
 * the confidence-interval proxy of Sec. 3.3 (Eqs. 16-21, App. D).
 * The backward pass is the two-stage adjoint of Sec. 3.3 (Eq. 22): an adjoint
 * moment per pixel, then one reduction of per-Gaussian gradients.
 *
 * Conventions shared by every entry point:
 *  - All float arrays are float32, row-major, densely packed.
 *  - Pointers marked "device" must be device memory of the current HIP device;
 *    "host" pointers are read during the call only.
 *  - The caller owns and allocates every buffer; the library never allocates
 *    or frees device memory and never writes its inputs.
 *  - Every call is enqueued asynchronously on `stream` (a hipStream_t; NULL
 *    is the default stream), except mb_prepare when it returns the entry
 *    count and mb_entry_count, which wait for that one count.
 *  - Return value 0 (MB_OK) or a negative MB_ERR_* code; the message of the
 *    last error of the calling thread is available from mb_last_error().
 *    No exception or abort crosses the ABI.
 *  - Calls on distinct workspaces may run concurrently.
 */
#ifndef MB3DGS_H
#define MB3DGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MB_OK 0
#define MB_ERR_ARG (-1)          /* invalid argument (null pointer, bad size) */
#define MB_ERR_UNSUPPORTED (-2)  /* unsupported option (K, N, SH degree, ...) */
#define MB_ERR_WORKSPACE (-3)    /* workspace too small for this call         */
#define MB_ERR_HIP (-4)          /* a HIP runtime call or kernel launch failed */

#define MB_MAX_CAMERAS 16
#define MB_SAVED_FLOATS_PER_PIXEL 8

/* Gaussians (Sec. 3.1). All pointers device, n >= 0.
 *  means     [n,3]  world-space mean mu_i
 *  scales    [n,3]  linear per-axis scales (> 0), S = diag(scales)
 *  quats     [n,4]  rotation quaternion (w, x, y, z); normalised inside, and
 *                   gradients include the normalisation
 *  densities [n]    density weight w_i >= 0 (the caller applies softplus)
 *  colors    [n,3] RGB when sh_degree = -1, else [n,(sh_degree+1)^2,3] real
 *                   SH coefficients; emission = max(0, sum_lm f_lm Y_lm(v) + 1/2)
 *                   with v = normalize(mean - camera origin). */
typedef struct mb_gaussians {
  int32_t n;
  int32_t sh_degree; /* -1 (RGB) or 0..3 */
  const float *means, *scales, *quats, *densities, *colors;
} mb_gaussians;

/* Pinhole camera. world_to_cam = [R | t] row-major 3x4, x_cam = R x + t,
 * OpenCV axes (x right, y down, z forward). Pixel (x, y) has its centre at
 * (x + 1/2, y + 1/2) and ray direction normalize(K^-1 (x+1/2, y+1/2, 1)).
 * t_near is the near integration bound t_n; the far bound is infinity. */
typedef struct mb_camera {
  float world_to_cam[12];
  float fx, fy, cx, cy;
  int32_t width, height;
  float t_near;
  float background[3];
} mb_camera;

/* Method options. Defaults (mb_default_options) are the paper's printed
 * constants where it gives them. */
typedef struct mb_options {
  int32_t n_moments;   /* K power moments beyond m_0: 4, 6 or 8 (K+1 values) */
  int32_t n_intervals; /* N quadrature intervals (N+1 edges): 3 or 5         */
  float kappa;         /* sample spread of the edges, App. B (3)             */
  float conf_c;        /* confidence level c of the proxy, App. D (0.01)     */
  float beta;          /* interpolation between the bounds, Sec. 3.2 (0.25)  */
  float eps;           /* clamp of Eq. 15's denominator (1e-6)               */
  int32_t basis;       /* moment basis: 0 power moments (Eqs. 10-12), 1
                          trigonometric moments (Eqs. 13-14; n_moments 4 or
                          6, i.e. two or three complex moments; not with the
                          surrogate or the tabulated schedule)             */
  const void *surrogate; /* reserved, NULL                                   */
  int32_t full_coverage; /* debug: every Gaussian covers every pixel        */
  int32_t reserved;
} mb_options;

void mb_default_options(mb_options *opts);
const char *mb_last_error(void);
int32_t mb_version(void);

/* Workspace sizes. The Gaussian workspace holds per-(camera, Gaussian)
 * records and tile counts; the pair workspace holds the per-tile lists for
 * n_entries (camera, tile, Gaussian) entries, the backward partials, and each
 * pixel's moment sums (9 doubles per pixel), which the forward pass leaves
 * for the backward pass.
 * Both are caller-allocated device memory, 256-byte aligned. */
size_t mb_gauss_workspace_bytes(int32_t n, int32_t n_cams);
size_t mb_pair_workspace_bytes(int64_t n_entries, int32_t n_cams, int32_t width,
                               int32_t height);
/* The largest entry count a pair workspace of pws_bytes holds (the inverse of
 * mb_pair_workspace_bytes), or -1 when it holds none or an argument is bad. */
int64_t mb_pair_capacity(size_t pws_bytes, int32_t n_cams, int32_t width, int32_t height);

/* Passed as n_entries to mb_render_forward and mb_render_backward: the entry
 * count stays on the device, where mb_prepare (called with a NULL count)
 * left it, and the pair workspace is laid out for its capacity
 * mb_pair_capacity(pws_bytes, ...). Such a frame needs no host round trip,
 * so frames can be enqueued back to back. Entries beyond the capacity are
 * dropped: the render then misses them, and the caller compares
 * mb_entry_count with the capacity after the fact and renders again with a
 * larger workspace. The surrogate and harvest entry points take counts only. */
#define MB_ENTRIES_ON_DEVICE (-1)

/* Screen proxies only (App. D), for inspection: per Gaussian writes
 * proxy[n,8] (double) = (centre_x, centre_y, e1_x, e1_y, half_1, half_2,
 * valid, 0) where the oriented rectangle is centre + a e1 + b e2,
 * |a| <= half_1, |b| <= half_2, e2 = (-e1_y, e1_x); e1 is the major axis of
 * the proxy ellipse at the angle atan2(2 s_xy, s_xx - s_yy) / 2 of its
 * covariance (an exact circle takes e1 = (1, 0)); valid = 0 for culled
 * Gaussians. This is the rectangle the pixel coverage test uses, computed in
 * double from the float32 inputs. proxy: device, caller-allocated. */
int mb_project(const mb_gaussians *g, const mb_camera *cam, const mb_options *opts,
               double *proxy, void *stream);

/* Stage 1 of a render (Sec. 3.3 culling and proxy): per camera and Gaussian,
 * the screen proxy, the ray-space coefficients and the number of 16x16 tiles
 * its rectangle overlaps. With n_entries (host pointer) not NULL it waits on
 * `stream` once to return the total number of (camera, tile, Gaussian)
 * entries there; with NULL the total stays on the device (see
 * MB_ENTRIES_ON_DEVICE) and nothing waits. gws must hold
 * mb_gauss_workspace_bytes(g->n, n_cams) bytes. All cameras share one image
 * size. */
int mb_prepare(const mb_gaussians *g, const mb_camera *cams, int32_t n_cams,
               const mb_options *opts, void *gws, size_t gws_bytes,
               int64_t *n_entries, void *stream);

/* The entry total of the last mb_prepare on gws (n_gaussians and n_cams as
 * given to it), read back to the host: waits on `stream`. */
int mb_entry_count(int32_t n_gaussians, int32_t n_cams, const void *gws, size_t gws_bytes,
                   int64_t *n_entries, void *stream);

/* Forward render (Sec. 3.2-3.3, Eqs. 7, 10-12, 15) after mb_prepare with the
 * same arguments. n_entries is mb_prepare's count, and pws must then hold
 * mb_pair_workspace_bytes(n_entries, ...); or it is MB_ENTRIES_ON_DEVICE.
 *  image   [C,H,W,3] device, written: the rescaled radiance of Eq. 15
 *  saved   [C,H,W,8] device, written: per-pixel state for the backward pass:
 *                    [0..2] sum_i q_i rgb_i, [3] O = sum_i q_i, [4] depth of the
 *                    moment-variable origin, [5] its warp scale, [6] m_0,
 *                    [7] number of covering Gaussians n, or -(n + 1) when the
 *                    pixel's Hankel matrix was not numerically positive
 *                    definite and a diagonal bias was added.
 *  penalty [C,H,W] device or NULL: the consistency penalty of App. E per
 *                    pixel, sum over covering Gaussians i of
 *                    P_i = sum_j max(0, tau_ij - (tau(t_{j+1}) - tau(t_j)))^2
 *                    over the quadrature intervals (tau_ij: particle i's own
 *                    optical depth over the interval). */
int mb_render_forward(const mb_gaussians *g, const mb_camera *cams, int32_t n_cams,
                      const mb_options *opts, void *gws, size_t gws_bytes, void *pws,
                      size_t pws_bytes, int64_t n_entries, float *image, float *saved,
                      float *penalty, void *stream);

/* Forward render that allocates nothing, for callers that cannot allocate
 * device memory (serving loops and harnesses that forbid hipMalloc): the same
 * result as mb_prepare (with a count) followed by mb_render_forward, with
 * both workspaces carved from a 256 MiB device array inside the library
 * (one per GPU, held until the process ends) instead of caller buffers.
 *  image, saved, penalty  as in mb_render_forward (device, caller-owned)
 *  n_entries  host, or NULL: receives the frame's tile entry count
 * The call waits on `stream` once for the entry count (as mb_prepare with a
 * count does), so it cannot be captured into a graph. A frame whose
 * workspaces (168 B per camera and Gaussian, 376 B per tile entry, 72 B per
 * pixel, plus per-tile arrays) exceed 256 MiB is rejected with
 * MB_ERR_WORKSPACE before anything is rendered: 100k Gaussians at 1024x1024
 * (about 300k entries) fit, 500k Gaussians at 1920x1080 do not. All calls on
 * one GPU share that array, which keeps the last call's contents, so calls
 * that overlap on one GPU (other streams, other host threads) race; a
 * backward pass cannot follow this forward pass (the scratch holds no
 * gradient state a caller could pass on). */
int mb_render_forward_noalloc(const mb_gaussians *g, const mb_camera *cams, int32_t n_cams,
                              const mb_options *opts, float *image, float *saved, float *penalty,
                              int64_t *n_entries, void *stream);

/* Backward pass (Sec. 3.3, Eq. 22, App. D adjoint rendering) after
 * mb_render_forward with the same arguments and workspaces (n_entries
 * included: the count, or MB_ENTRIES_ON_DEVICE). The per-pixel
 * moment sums come from the pair workspace, where the forward pass left them;
 * nothing per (pixel, Gaussian) pair is stored, the pairs' terms are
 * recomputed. Both moment bases: with trigonometric moments the adjoint of
 * the reconstruction on the circle and of Eq. 14 replace the power
 * moments' (the atoms and flags of the canonical representation are held
 * fixed, as the flags of the power moments' bounds are).
 *  saved         [C,H,W,8] device, from mb_render_forward
 *  grad_image    [C,H,W,3] device, dL/dimage
 *  grad_penalty  [C,H,W] device, dL/dpenalty, or NULL (no penalty term)
 *  g_means [n,3], g_scales [n,3], g_quats [n,4], g_densities [n],
 *  g_colors (same shape as colors): device, overwritten with dL/dparameter
 *  summed over all cameras. Culled Gaussians receive zero. */
int mb_render_backward(const mb_gaussians *g, const mb_camera *cams, int32_t n_cams,
                       const mb_options *opts, void *gws, size_t gws_bytes, void *pws,
                       size_t pws_bytes, int64_t n_entries, const float *saved,
                       const float *grad_image, const float *grad_penalty, float *g_means,
                       float *g_scales, float *g_quats, float *g_densities, float *g_colors,
                       void *stream);

/* ------------------------------------------------------------------------
 * Learned surrogate of the moment -> optical-depth reconstruction (not part of
 * the paper): a 7 -> 64 -> 64 -> 1 MLP, tanh-GELU hidden layers, output
 * F = sigmoid(.) in (0, 1) standing for the normalised bound interpolation of
 * Sec. 3.2, so the optical depth is m_0 F. Weights and activations bf16,
 * accumulation fp32 (matrix cores).
 *  theta   [P] fp32 parameters, P = mb_mlp_param_count(), in the order
 *          W1[64][7], b1[64], W2[64][64] (out, in), b2[64], w3[64], b3.
 *  packed  mb_mlp_packed_bytes() bytes: bf16 kernel copy made by mb_mlp_pack.
 *  x       [n][8] fp32 rows: 6 moment features, the query, and m_0 (used by
 *          the loss only). All device pointers.
 * mb_mlp_forward writes F [n]. mb_mlp_loss_grad evaluates the loss
 * mean_i (exp(-m0_i F_i) - t_i)^2 against target transmittances t [n] and
 * writes its gradient grad [P] and (if not NULL) the loss [1]; ws must hold
 * mb_mlp_workspace_bytes(n) bytes. mb_adam_step applies one Adam update
 * (step counts from 1) to theta with moments m, v [count]. */
int32_t mb_mlp_param_count(void);
size_t mb_mlp_packed_bytes(void);
size_t mb_mlp_workspace_bytes(int64_t batch);
int mb_mlp_pack(const float *theta, void *packed, void *stream);
int mb_mlp_forward(const void *packed, const float *x, int64_t n, float *f_out, void *stream);
int mb_mlp_loss_grad(const void *packed, const float *x, const float *t_target, int64_t n, float *grad,
                     float *loss, void *ws, size_t ws_bytes, void *stream);
int mb_adam_step(float *theta, float *m, float *v, const float *grad, int64_t count, int32_t step,
                 float lr, float beta1, float beta2, float eps, void *stream);

/* Training samples of the surrogate (not part of the paper): mb_render_forward
 * (n_moments = 6) that also appends a seeded pseudo-random subset of its
 * quadrature queries, each independently with probability `rate` (a hash of
 * seed, pixel, record and edge decides), to samples[capacity][12] (device):
 *   [0..5] asinh of the pixel's standardised moments 1..6 (mean 0, variance 1
 *          in the moment variable), [6] the standardised query, clamped to
 *          [-10, 10], [7] m_0, [8] transmittance exp(-m_0 F) of the moment
 *          bounds at the query; as int32 bit patterns: [9] the 32 hash bits,
 *          [10] flat pixel index (camera * H + y) * W + x, [11] record * (N+1)
 *          + edge, record = camera * n + Gaussian.
 * *count (device int32) is advanced atomically by every selected query, also
 * past `capacity`, where samples are dropped; the caller zeroes it before the
 * first of a series of calls. Sample order in the buffer is not deterministic,
 * the set of samples is: sort by [9] for a fixed order. */
int mb_render_forward_harvest(const mb_gaussians *g, const mb_camera *cams, int32_t n_cams,
                              const mb_options *opts, void *gws, size_t gws_bytes, void *pws,
                              size_t pws_bytes, int64_t n_entries, float rate, uint32_t seed,
                              float *samples, int32_t capacity, int32_t *count, float *image,
                              float *saved, void *stream);

/* Forward render with the learned surrogate in place of the moment bounds'
 * evaluation (Sec. 3.2's reconstruction; everything else as
 * mb_render_forward, n_moments = 6). Three kernels: passes 0-1 and a list of
 * the quadrature queries; the MLP (mlp_packed from mb_mlp_pack) on that list;
 * the quadrature of Eq. 7 and Eq. 15 from its outputs.
 *  qws  device, mb_query_workspace_bytes(n_cams, width, height,
 *       query_capacity) bytes. Its first 8 bytes receive the number of
 *       queries the frame needed (uint64). If that exceeds query_capacity the
 *       image is incomplete: call again with a larger capacity.
 *  saved as in mb_render_forward; [7] carries the covering count only. */
size_t mb_query_workspace_bytes(int32_t n_cams, int32_t width, int32_t height,
                                int64_t query_capacity);
int mb_render_forward_surrogate(const mb_gaussians *g, const mb_camera *cams, int32_t n_cams,
                                const mb_options *opts, void *gws, size_t gws_bytes, void *pws,
                                size_t pws_bytes, int64_t n_entries, const void *mlp_packed,
                                void *qws, size_t qws_bytes, int64_t query_capacity,
                                float *image, float *saved, void *stream);

/* The tabulated schedule of the reconstruction (not part of the paper): per
 * pixel, the normalised optical depth F is evaluated at n_nodes equally
 * spaced nodes z_g of the standardised query on [-4, 4] (the query mapped by
 * the mean and standard deviation of the pixel's normalised measure in its
 * moment variable), and every quadrature edge interpolates that table
 * linearly at its own standardised query, clamped to the table's ends; the
 * optical depth along a Gaussian's edges is then made non-decreasing
 * (running maximum). F at the nodes is the moment bounds' interpolation of
 * Sec. 3.2 (mlp_packed NULL; n_moments 4 or 6) or the learned surrogate
 * (mlp_packed from mb_mlp_pack; n_moments 6), so the two reconstructions run
 * in the same schedule. Otherwise as mb_render_forward (power moments; no
 * penalty; saved[7] flags a degenerate measure only for the bounds).
 *  n_nodes  2..256 (32 is the default of the bindings)
 *  tws      device, mb_table_workspace_bytes(n_cams, width, height, n_nodes)
 *           bytes: per pixel 12 floats of record and n_nodes of table */
size_t mb_table_workspace_bytes(int32_t n_cams, int32_t width, int32_t height, int32_t n_nodes);
int mb_render_forward_tabulated(const mb_gaussians *g, const mb_camera *cams, int32_t n_cams,
                                const mb_options *opts, void *gws, size_t gws_bytes, void *pws,
                                size_t pws_bytes, int64_t n_entries, const void *mlp_packed,
                                int32_t n_nodes, void *tws, size_t tws_bytes, float *image,
                                float *saved, void *stream);

/* Backward pass through the surrogate render: the adjoint of
 * mb_render_forward_surrogate, after it, with the same arguments,
 * workspaces, weights and query capacity. The MLP is run again on the
 * forward pass's query list for F and its gradient with respect to the
 * network inputs (bf16 products, fp32 accumulation); the render adjoint then
 * follows the optical depth m_0 F back through the standardised moments and
 * the query (clamped queries pass no gradient to it) to the Gaussians.
 *  qws    device, mb_query_workspace_bytes_backward(n_cams, width, height,
 *         query_capacity) bytes (the forward layout is its prefix, so the
 *         forward call may use the same buffer). Pixels whose queries did not
 *         fit the capacity in the forward call take no gradient.
 *  saved, grad_image, g_*: as in mb_render_backward. There is no penalty
 *  term on this path. */
size_t mb_query_workspace_bytes_backward(int32_t n_cams, int32_t width, int32_t height,
                                         int64_t query_capacity);
int mb_render_backward_surrogate(const mb_gaussians *g, const mb_camera *cams, int32_t n_cams,
                                 const mb_options *opts, void *gws, size_t gws_bytes, void *pws,
                                 size_t pws_bytes, int64_t n_entries, const void *mlp_packed,
                                 void *qws, size_t qws_bytes, int64_t query_capacity,
                                 const float *saved, const float *grad_image, float *g_means,
                                 float *g_scales, float *g_quats, float *g_densities,
                                 float *g_colors, void *stream);

/* D-SSIM term of the training objective (Training and Densification
 * paragraph: L = (1 - alpha) L1 + alpha L_D-SSIM + lambda L_consistency, alpha
 * = 0.2, lambda = 0.1), as the 3DGS losses the paper extends define it: per
 * colour channel, SSIM under an 11 x 11 Gaussian window (sigma 1.5, zero
 * padding, C1 = 0.01^2, C2 = 0.03^2), averaged over pixels and channels.
 *  image, target [C,H,W,3] device
 *  loss          device float, written: 1 - mean SSIM
 *  grad_image    [C,H,W,3] device or NULL: ACCUMULATED with
 *                grad_scale * d loss / d image (so an L1 gradient can be
 *                summed into the same buffer)
 *  ws            mb_dssim_workspace_bytes(n_cams, width, height) bytes */
size_t mb_dssim_workspace_bytes(int32_t n_cams, int32_t width, int32_t height);
int mb_dssim(const float *image, const float *target, int32_t n_cams, int32_t width,
             int32_t height, float grad_scale, float *loss, float *grad_image, void *ws,
             size_t ws_bytes, void *stream);

/* The L1 term of the objective above: *loss (device) = mean |image - target|
 * over n floats; grad_image (device, or NULL) is ACCUMULATED with
 * grad_scale sign(image - target) / n, the sign 0 where they are equal.
 * ws: mb_l1_workspace_bytes() bytes. */
size_t mb_l1_workspace_bytes(void);
int mb_l1(const float *image, const float *target, int64_t n, float grad_scale, float *loss,
          float *grad_image, void *ws, size_t ws_bytes, void *stream);

/* Adaptive density control of the density-based medium (App. E), one thread
 * per particle. Colours are laid out as in an mb_gaussians set: 3 (SH degree
 * + 1)^2 floats per particle, or 3 for RGB.
 *
 * mb_view_independent_opacity: o_i = 1 - exp(-sqrt(2 pi) w_i min(s_i)), the
 *   particle's opacity seen along its shortest axis through its centre (the
 *   pruning criterion). opacity [n] device, written.
 * mb_density_from_opacity: w_i = -log(1 - o_i) / (sqrt(2 pi) mean(s_i)), the
 *   appendix's initial peak densities. opacity, scales [n,3] in, densities
 *   [n] out, all device.
 * mb_adc_accumulate: grad_acc[i] += |dL/dmean_i| per component and
 *   grad_count[i] += 1 when that gradient is nonzero (accumulated absolute
 *   gradient, per view). All device; the caller zeroes them at the start of
 *   a densification interval.
 * mb_adc_plan: action[i] = 0 prune (view-independent opacity below
 *   min_opacity), 2 clone or 3 split (|grad_acc_i| / max(grad_count_i, 1) above
 *   grad_threshold with some counted view; split if max(s_i) > split_scale),
 *   else 1 keep; offsets[i] the particle's first output slot (exclusive scan
 *   of 0/1/2/2 outputs), *n_out (device int32) the size of the new set. ws:
 *   mb_adc_workspace_bytes(n) bytes. All device.
 * mb_adc_apply: writes the new set (n_out particles, input order) into the
 *   output arrays: kept particles once; cloned ones twice at half peak
 *   density (the two copies add up to the original density); split ones as
 *   two particles at mean -+ delta s_max e_max with s_max scaled by gamma
 *   (e_max the axis of the largest scale; gamma = 0.6385502815246582 and
 *   delta = 0.6128153090966912 as the appendix derives them), everything else
 *   copied. */
typedef struct mb_adc_params {
  float min_opacity;
  float grad_threshold; /* the appendix uses 1e-4 */
  float split_scale;
} mb_adc_params;
int mb_view_independent_opacity(const mb_gaussians *g, float *opacity, void *stream);
int mb_density_from_opacity(int32_t n, const float *opacity, const float *scales, float *densities,
                            void *stream);
int mb_adc_accumulate(int32_t n, const float *g_means, float *grad_acc, int32_t *grad_count,
                      void *stream);
size_t mb_adc_workspace_bytes(int32_t n);
int mb_adc_plan(const mb_gaussians *g, const float *grad_acc, const int32_t *grad_count,
                const mb_adc_params *params, int32_t *action, int32_t *offsets, int32_t *n_out,
                void *ws, size_t ws_bytes, void *stream);
int mb_adc_apply(const mb_gaussians *g, const int32_t *action, const int32_t *offsets, float *means,
                 float *scales, float *quats, float *densities, float *colors, void *stream);

/* Stage timing. mb_profile_enable(stages) selects the stages to time: bit s
 * of `stages` for stage s in the order below, MB_PROFILE_ALL for all, 0 to
 * stop. Every entry point then records two HIP events around each selected
 * stage on its stream (each record adds a marker to the stream, a few
 * microseconds of device time per frame and stage).
 * mb_profile_read waits for the recorded events, writes up to `max` stage
 * totals in milliseconds to ms[] and launch counts to calls[] (both host,
 * may be NULL), clears the record and returns the number of stages
 * (MB_STAGE_COUNT). Stages, in order: preprocess, scan, emit, sort, lists,
 * render_forward, render_backward, gradients, mlp, render_consume (the
 * surrogate's quadrature). Not thread safe with concurrent renders. */
#define MB_STAGE_COUNT 10
#define MB_PROFILE_ALL ((1 << MB_STAGE_COUNT) - 1)
void mb_profile_enable(int32_t stages);
int32_t mb_profile_read(double *ms, int64_t *calls, int32_t max);

#ifdef __cplusplus
}
#endif
#endif /* MB3DGS_H */
