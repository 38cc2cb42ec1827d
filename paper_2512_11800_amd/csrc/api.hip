// C ABI of the rendering path: argument checks, workspace layout and the
// launch sequence of each entry point (see include/mb3dgs.h).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"

using namespace mb;

namespace {

// ---------------------------------------------------------------------------
// Stage timing with HIP events on the caller's stream (mb_profile_*).
// ---------------------------------------------------------------------------
enum Stage { S_PREPROCESS = 0, S_SCAN, S_EMIT, S_SORT, S_LISTS, S_RENDER_FWD, S_RENDER_BWD, S_GRADS, S_MLP, S_CONSUME };

struct Profiler {
  std::mutex mu;
  uint32_t mask = 0;  // stages being timed (bit s for stage s)
  struct Rec { int stage; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
Profiler g_prof;

struct StageTimer {
  int stage;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  StageTimer(int st, hipStream_t str) : stage(st), s(str) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    if (!((g_prof.mask >> stage) & 1u)) return;
    a = g_prof.get();
    b = g_prof.get();
    if (a && b && hipEventRecord(a, s) == hipSuccess) return;
    release();  // no timing for this stage
  }
  ~StageTimer() {
    if (!a || !b) return;
    const bool ok = hipEventRecord(b, s) == hipSuccess;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    if (ok) g_prof.recs.push_back({stage, a, b});
    else release();
  }
  // hand the events back to the pool (g_prof.mu held)
  void release() {
    if (a) g_prof.pool.push_back(a);
    if (b) g_prof.pool.push_back(b);
    a = b = nullptr;
  }
};

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(MB_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Carves consecutive 256-byte aligned regions out of a workspace.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* p) : base(static_cast<char*>(p)) {}
  template <class T>
  T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off = align_up(off + count * sizeof(T));
    return p;
  }
};

struct GaussWs {
  float4* rec;
  double2* rectd;
  int4* tbox;
  int* counts;
  int* offsets;
  int* scan_tmp;
  int* total;
  size_t bytes;
};

GaussWs carve_gauss(void* p, int64_t n, int n_cams) {
  Carver c(p);
  int64_t m = n * n_cams;
  GaussWs w;
  w.rec = c.take<float4>((size_t)m * kRecStride);
  w.rectd = c.take<double2>((size_t)m * 3);
  w.tbox = c.take<int4>((size_t)m);
  w.counts = c.take<int>((size_t)m);
  w.offsets = c.take<int>((size_t)m);
  w.scan_tmp = c.take<int>(scan_tmp_ints(m));
  w.total = c.take<int>(1);
  w.bytes = c.off;
  return w;
}

struct PairWs {
  uint32_t *keys_a, *keys_b;
  int *vals_a, *vals_b, *entry_rec, *sorted_rec, *radix_tmp;
  int2* ranges;
  int *order, *order_tmp;
  uint64_t* masks;
  float* partials;
  uint8_t* used;  // [E,4]: the backward wrote slot (entry, wave)
  double* pix_mom;
  size_t bytes;
};

PairWs carve_pairs(void* p, int64_t e, int n_keys, int64_t n_pix) {
  Carver c(p);
  PairWs w;
  w.keys_a = c.take<uint32_t>((size_t)e);
  w.keys_b = c.take<uint32_t>((size_t)e);
  w.vals_a = c.take<int>((size_t)e);
  w.vals_b = c.take<int>((size_t)e);
  w.entry_rec = c.take<int>((size_t)e);
  w.sorted_rec = c.take<int>((size_t)e);
  w.radix_tmp = c.take<int>(radix_tmp_ints(e));
  w.ranges = c.take<int2>((size_t)n_keys);
  w.order = c.take<int>((size_t)render_blocks(n_keys));
  w.order_tmp = c.take<int>(order_tmp_ints(n_keys));
  w.masks = c.take<uint64_t>((size_t)e * 4);
  w.partials = c.take<float>((size_t)e * 4 * kGradStride);  // one slot per (entry, wave)
  w.used = c.take<uint8_t>((size_t)e * 4);
  w.pix_mom = c.take<double>((size_t)n_pix * (kMaxMoments + 1));
  w.bytes = c.off;
  return w;
}

int tiles_of(int px) { return (px + kTile - 1) / kTile; }

// largest entry count whose pair workspace fits in `bytes` (-1: none)
int64_t pair_capacity(size_t bytes, int n_cams, int width, int height) {
  const int n_keys = tiles_of(width) * tiles_of(height) * n_cams;
  const int64_t n_pix = (int64_t)n_cams * width * height;
  if (carve_pairs(nullptr, 0, n_keys, n_pix).bytes > bytes) return -1;
  int64_t lo = 0, hi = INT32_MAX;  // entry indices are int
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (carve_pairs(nullptr, mid, n_keys, n_pix).bytes <= bytes) lo = mid; else hi = mid - 1;
  }
  return lo;
}

int check_common(const mb_gaussians* g, const mb_camera* cams, int n_cams, const mb_options* o) {
  if (!g || !cams || !o) return fail(MB_ERR_ARG, "null gaussians, cameras or options");
  if (g->n < 0) return fail(MB_ERR_ARG, "negative Gaussian count %d", g->n);
  if (g->n > 0 && (!g->means || !g->scales || !g->quats || !g->densities || !g->colors))
    return fail(MB_ERR_ARG, "null Gaussian parameter pointer");
  if (g->sh_degree < -1 || g->sh_degree > 3) return fail(MB_ERR_UNSUPPORTED, "SH degree %d not in -1..3", g->sh_degree);
  if (n_cams < 1 || n_cams > MB_MAX_CAMERAS) return fail(MB_ERR_ARG, "camera count %d not in 1..%d", n_cams, MB_MAX_CAMERAS);
  for (int i = 0; i < n_cams; ++i) {
    const mb_camera& c = cams[i];
    if (c.width <= 0 || c.height <= 0 || c.width > 16384 || c.height > 16384)
      return fail(MB_ERR_ARG, "camera %d: image size %dx%d out of range", i, c.width, c.height);
    if (c.width != cams[0].width || c.height != cams[0].height)
      return fail(MB_ERR_ARG, "camera %d: all cameras must share one image size", i);
    if (!(c.fx > 0.f) || !(c.fy > 0.f) || !(c.t_near > 0.f))
      return fail(MB_ERR_ARG, "camera %d: focal lengths and t_near must be positive", i);
  }
  if (o->n_moments != 4 && o->n_moments != 6 && o->n_moments != 8)
    return fail(MB_ERR_UNSUPPORTED, "n_moments %d: only 4, 6 and 8", o->n_moments);
  if (o->n_intervals != 3 && o->n_intervals != 5)
    return fail(MB_ERR_UNSUPPORTED, "n_intervals %d: only 3 and 5", o->n_intervals);
  if (!(o->conf_c > 0.f && o->conf_c < 1.f)) return fail(MB_ERR_ARG, "conf_c must be in (0, 1)");
  if (!(o->kappa >= 1.f)) return fail(MB_ERR_ARG, "kappa must be >= 1");
  if (!(o->eps > 0.f)) return fail(MB_ERR_ARG, "eps must be positive");
  if (o->basis != 0 && o->basis != 1) return fail(MB_ERR_ARG, "basis %d: 0 (power) or 1 (trigonometric)", o->basis);
  if (o->basis == 1 && o->n_moments != 4 && o->n_moments != 6)
    return fail(MB_ERR_UNSUPPORTED, "trigonometric moments: n_moments 4 or 6 (two or three complex moments)");
  int64_t keys = (int64_t)tiles_of(cams[0].width) * tiles_of(cams[0].height) * n_cams;
  if (keys >= (1ll << 30)) return fail(MB_ERR_ARG, "too many tiles");
  if ((int64_t)g->n * n_cams >= (1ll << 31)) return fail(MB_ERR_ARG, "too many Gaussian-camera pairs");
  return MB_OK;
}

CamSet make_cams(const mb_camera* cams, int n_cams) {
  CamSet s;
  memset(&s, 0, sizeof(s));
  s.n_cams = n_cams;
  for (int i = 0; i < n_cams; ++i) {
    const mb_camera& m = cams[i];
    CamConst& c = s.c[i];
    for (int r = 0; r < 3; ++r) {
      for (int k = 0; k < 3; ++k) c.r[r * 3 + k] = m.world_to_cam[r * 4 + k];
      c.t[r] = m.world_to_cam[r * 4 + 3];
    }
    for (int k = 0; k < 3; ++k) {  // origin = -R^T t
      double o = 0.0;
      for (int r = 0; r < 3; ++r) o -= (double)c.r[r * 3 + k] * (double)c.t[r];
      c.o[k] = (float)o;
    }
    c.fx = m.fx; c.fy = m.fy; c.cx = m.cx; c.cy = m.cy; c.tn = m.t_near;
    for (int k = 0; k < 3; ++k) c.bg[k] = m.background[k];
    c.width = m.width; c.height = m.height;
  }
  return s;
}

double conf_term(float c) { return std::log(-std::log1p(-(double)c) / std::sqrt(2.0 * M_PI)); }

// Standard-normal quantile by Newton's method on the normal CDF
// Phi(x) = erfc(-x / sqrt2) / 2 (App. B sample spacing).
double normal_quantile(double u) {
  double x = 0.0;
  for (int it = 0; it < 100; ++it) {
    double f = 0.5 * std::erfc(-x / std::sqrt(2.0)) - u;
    double d = std::exp(-0.5 * x * x) / std::sqrt(2.0 * M_PI);
    double step = f / d;
    x -= step;
    if (std::fabs(step) < 1e-15 * (1.0 + std::fabs(x))) break;
  }
  return x;
}

void fill_quantiles(const mb_options* o, float* xq, float* eq, float* ecq) {
  int nq = o->n_intervals + 1;
  for (int j = 0; j < 8; ++j) { xq[j] = 0.f; eq[j] = 0.f; ecq[j] = 0.f; }
  for (int j = 0; j < nq; ++j) {
    // midpoint reading of the uniformly spaced samples of App. B
    double x = normal_quantile((j + 0.5) / nq);
    xq[j] = (float)x;
    eq[j] = (float)std::exp(-0.5 * (double)o->kappa * o->kappa * x * x);
    ecq[j] = (float)std::erfc((double)o->kappa * x / std::sqrt(2.0));
  }
}

int key_bits(int64_t n_keys) {
  int b = 1;
  while ((1ll << b) < n_keys) ++b;
  return b;
}

// emit, sort and per-tile lists of the forward entry points
// n_entries: the list count, or (with n_dev) the capacity the launches are
// sized for, the count itself read on the device
int build_lists(const mb_gaussians* g, const GaussWs& w, const PairWs& p, int n_cams, int tx, int ty,
                int full_coverage, int64_t n_entries, const int* n_dev, hipStream_t s, bool split_heavy = true) {
  int n_keys = tx * ty * n_cams;
  EmitArgs ea;
  ea.rec = w.rec; ea.tbox = w.tbox; ea.offsets = w.offsets; ea.counts = w.counts;
  ea.n = g->n; ea.n_cams = n_cams; ea.tiles_x = tx; ea.tiles_y = ty; ea.full_coverage = full_coverage;
  ea.keys = p.keys_a; ea.entry_rec = p.entry_rec;
  ea.ranges = g->n > 0 ? p.ranges : nullptr;  // no emit launch without Gaussians
  ea.n_keys = n_keys;
  ea.cap = n_entries;
  hipError_t e;
  {
    StageTimer t(S_EMIT, s);
    e = launch_emit(ea, s);
  }
  if (e != hipSuccess) return hip_fail(e, "emit");
  {
    StageTimer t(S_SORT, s);
    e = launch_radix_sort(p.keys_a, p.vals_a, p.keys_b, p.vals_b, n_entries, n_dev, key_bits(n_keys), p.radix_tmp,
                          s, true);
  }
  if (e != hipSuccess) return hip_fail(e, "sort");
  {
    StageTimer t(S_LISTS, s);
    e = launch_finish_lists(p.keys_a, p.vals_a, p.entry_rec, n_entries, n_dev, p.sorted_rec, p.ranges, n_keys,
                            ea.ranges != nullptr, s);
    if (e == hipSuccess)
      e = launch_tile_order(p.ranges, n_keys, split_heavy ? kSplitEntries : 0x7FFFFFFF, p.order, p.order_tmp, s);
  }
  if (e != hipSuccess) return hip_fail(e, "lists");
  return MB_OK;
}

struct FwdSetup {
  GaussWs w;
  PairWs p;
  CamSet cs;
  RenderArgs ra;
  int n_keys;
  int64_t cap;       // list entries the pair workspace is laid out for
  const int* n_dev;  // the count on the device (MB_ENTRIES_ON_DEVICE), else null
};

// argument and workspace checks shared by the forward entry points
int forward_setup(const mb_gaussians* g, const mb_camera* cams, int32_t n_cams, const mb_options* o, void* gws,
                  size_t gws_bytes, void* pws, size_t pws_bytes, int64_t n_entries, float* image, float* saved,
                  FwdSetup& f, bool device_count_ok = false) {
  int rc = check_common(g, cams, n_cams, o);
  if (rc) return rc;
  if (!image || !saved) return fail(MB_ERR_ARG, "null image or saved output");
  if (n_entries < 0 && !(device_count_ok && n_entries == MB_ENTRIES_ON_DEVICE))
    return fail(MB_ERR_ARG, "n_entries %lld is neither a count nor accepted here as MB_ENTRIES_ON_DEVICE",
                (long long)n_entries);
  f.w = carve_gauss(gws, g->n, n_cams);
  if (!gws || gws_bytes < f.w.bytes)
    return fail(MB_ERR_WORKSPACE, "Gaussian workspace needs %zu bytes, got %zu", f.w.bytes, gws_bytes);
  int tx = tiles_of(cams[0].width), ty = tiles_of(cams[0].height);
  f.n_keys = tx * ty * n_cams;
  f.n_dev = nullptr;
  f.cap = n_entries;
  if (n_entries == MB_ENTRIES_ON_DEVICE) {
    f.cap = pws ? pair_capacity(pws_bytes, n_cams, cams[0].width, cams[0].height) : -1;
    if (f.cap < 0) return fail(MB_ERR_WORKSPACE, "pair workspace of %zu bytes holds no list", pws_bytes);
    f.n_dev = f.w.total;
  }
  f.p = carve_pairs(pws, f.cap, f.n_keys, (int64_t)n_cams * cams[0].width * cams[0].height);
  if (!pws || pws_bytes < f.p.bytes)
    return fail(MB_ERR_WORKSPACE, "pair workspace needs %zu bytes, got %zu", f.p.bytes, pws_bytes);
  f.cs = make_cams(cams, n_cams);
  RenderArgs& ra = f.ra;
  memset(&ra, 0, sizeof(ra));
  ra.rec = f.w.rec; ra.rectd = f.w.rectd; ra.sorted_rec = f.p.sorted_rec; ra.ranges = f.p.ranges; ra.order = f.p.order;
  ra.masks = f.p.masks;
  ra.pix_mom = f.p.pix_mom;
  ra.n_pix = (long long)n_cams * cams[0].width * cams[0].height;
  ra.image = image; ra.saved = saved;
  ra.tiles_x = tx; ra.tiles_y = ty; ra.n_cams = n_cams; ra.full_coverage = o->full_coverage;
  ra.kappa = o->kappa; ra.beta = o->beta; ra.eps = o->eps;
  fill_quantiles(o, ra.xq, ra.eq, ra.ecq);
  return MB_OK;
}

struct QueryWs {
  unsigned long long* count;
  float* pixfeat;
  long long* pix_qbase;
  float *q_z, *q_f;
  int* q_pix;
  float* q_g;  // backward only: F and dF/d(inputs) per query, [q][8]
  size_t bytes;
};

// The forward layout is a prefix of the backward one, so a workspace sized
// for the backward pass serves both.
QueryWs carve_queries(void* p, int64_t n_pix, int64_t q_cap, bool grads = false) {
  Carver c(p);
  QueryWs w;
  w.count = c.take<unsigned long long>(1);
  w.pixfeat = c.take<float>((size_t)n_pix * kPixFeat);
  w.pix_qbase = c.take<long long>((size_t)n_pix);
  w.q_z = c.take<float>((size_t)q_cap);
  w.q_pix = c.take<int>((size_t)q_cap);
  w.q_f = c.take<float>((size_t)q_cap);
  w.q_g = grads ? c.take<float>((size_t)q_cap * 8) : nullptr;
  w.bytes = c.off;
  return w;
}

}  // namespace

// ---------------------------------------------------------------------------
// Device scratch of mb_render_forward_noalloc: the Gaussian and pair
// workspaces of one forward frame, in a file-scope device array (each GPU the
// library runs on holds its own copy until the process ends). Host code uses
// the address hipGetSymbolAddress returns for the current device, never the
// array's name.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// the current device's scratch address, looked up once per device
int scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(MB_ERR_ARG, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MB_OK;
}
}  // namespace

extern "C" {

void mb_default_options(mb_options* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->n_moments = 4;
  o->n_intervals = 3;
  o->kappa = 3.f;
  o->conf_c = 0.01f;
  o->beta = 0.25f;
  o->eps = 1e-6f;
}

const char* mb_last_error(void) { return g_err.c_str(); }

void mb_profile_enable(int32_t stages) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.mask = (uint32_t)stages & ((1u << MB_STAGE_COUNT) - 1u);
}

int32_t mb_profile_read(double* ms, int64_t* calls, int32_t max) {
  std::vector<Profiler::Rec> recs;
  {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    recs.swap(g_prof.recs);
  }
  double tot[MB_STAGE_COUNT] = {0};
  int64_t cnt[MB_STAGE_COUNT] = {0};
  for (auto& r : recs) {
    float t = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
      tot[r.stage] += t;
      cnt[r.stage] += 1;
    }
  }
  {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    for (auto& r : recs) { g_prof.pool.push_back(r.a); g_prof.pool.push_back(r.b); }
  }
  for (int i = 0; i < MB_STAGE_COUNT && i < max; ++i) {
    if (ms) ms[i] = tot[i];
    if (calls) calls[i] = cnt[i];
  }
  return MB_STAGE_COUNT;
}

int32_t mb_version(void) { return 1; }

size_t mb_gauss_workspace_bytes(int32_t n, int32_t n_cams) {
  if (n < 0 || n_cams < 1) return 0;
  return carve_gauss(nullptr, n, n_cams).bytes;
}

size_t mb_pair_workspace_bytes(int64_t n_entries, int32_t n_cams, int32_t width, int32_t height) {
  if (n_entries < 0 || n_cams < 1 || width <= 0 || height <= 0) return 0;
  int n_keys = tiles_of(width) * tiles_of(height) * n_cams;
  return carve_pairs(nullptr, n_entries, n_keys, (int64_t)n_cams * width * height).bytes;
}

int64_t mb_pair_capacity(size_t pws_bytes, int32_t n_cams, int32_t width, int32_t height) {
  if (n_cams < 1 || width <= 0 || height <= 0) return -1;
  return pair_capacity(pws_bytes, n_cams, width, height);
}

int mb_entry_count(int32_t n_gaussians, int32_t n_cams, const void* gws, size_t gws_bytes, int64_t* n_entries,
                   void* stream) {
  if (n_gaussians < 0 || n_cams < 1 || !n_entries) return fail(MB_ERR_ARG, "bad arguments");
  GaussWs w = carve_gauss(const_cast<void*>(gws), n_gaussians, n_cams);
  if (!gws || gws_bytes < w.bytes)
    return fail(MB_ERR_WORKSPACE, "Gaussian workspace needs %zu bytes, got %zu", w.bytes, gws_bytes);
  hipStream_t s = (hipStream_t)stream;
  int total = 0;
  hipError_t e = hipMemcpyAsync(&total, w.total, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "count readback");
  if (total < 0) return fail(MB_ERR_ARG, "tile entry count overflow");
  *n_entries = total;
  return MB_OK;
}

int mb_project(const mb_gaussians* g, const mb_camera* cam, const mb_options* o, double* proxy, void* stream) {
  int rc = check_common(g, cam, 1, o);
  if (rc) return rc;
  if (g->n > 0 && !proxy) return fail(MB_ERR_ARG, "null proxy output");
  PrepArgs a;
  memset(&a, 0, sizeof(a));
  a.means = g->means; a.scales = g->scales; a.quats = g->quats; a.dens = g->densities; a.colors = g->colors;
  a.n = g->n; a.sh_degree = g->sh_degree;
  a.tiles_x = tiles_of(cam->width); a.tiles_y = tiles_of(cam->height);
  a.conf_term = conf_term(o->conf_c);
  a.full_coverage = o->full_coverage;
  a.proxy_out = proxy;
  CamSet cs = make_cams(cam, 1);
  hipError_t e = launch_preprocess(a, cs, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "mb_project");
  return MB_OK;
}

int mb_prepare(const mb_gaussians* g, const mb_camera* cams, int32_t n_cams, const mb_options* o, void* gws,
               size_t gws_bytes, int64_t* n_entries, void* stream) {
  int rc = check_common(g, cams, n_cams, o);
  if (rc) return rc;
  GaussWs w = carve_gauss(gws, g->n, n_cams);
  if (!gws || gws_bytes < w.bytes)
    return fail(MB_ERR_WORKSPACE, "Gaussian workspace needs %zu bytes, got %zu", w.bytes, gws_bytes);
  hipStream_t s = (hipStream_t)stream;
  PrepArgs a;
  memset(&a, 0, sizeof(a));
  a.means = g->means; a.scales = g->scales; a.quats = g->quats; a.dens = g->densities; a.colors = g->colors;
  a.n = g->n; a.sh_degree = g->sh_degree;
  a.tiles_x = tiles_of(cams[0].width); a.tiles_y = tiles_of(cams[0].height);
  a.conf_term = conf_term(o->conf_c);
  a.full_coverage = o->full_coverage;
  a.rec = w.rec; a.rectd = w.rectd; a.tbox = w.tbox; a.counts = w.counts;
  CamSet cs = make_cams(cams, n_cams);
  hipError_t e;
  {
    StageTimer t(S_PREPROCESS, s);
    e = launch_preprocess(a, cs, s);
  }
  if (e != hipSuccess) return hip_fail(e, "preprocess");
  {
    StageTimer t(S_SCAN, s);
    e = launch_scan(w.counts, w.offsets, (int64_t)g->n * n_cams, w.scan_tmp, w.total, s);
  }
  if (e != hipSuccess) return hip_fail(e, "scan");
  if (!n_entries) return MB_OK;  // the count stays on the device
  int total = 0;
  e = hipMemcpyAsync(&total, w.total, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_fail(e, "count readback");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "count readback sync");
  if (total < 0) return fail(MB_ERR_ARG, "tile entry count overflow");
  *n_entries = total;
  return MB_OK;
}

int mb_render_forward(const mb_gaussians* g, const mb_camera* cams, int32_t n_cams, const mb_options* o, void* gws,
                      size_t gws_bytes, void* pws, size_t pws_bytes, int64_t n_entries, float* image, float* saved,
                      float* penalty, void* stream) {
  FwdSetup f;
  int rc = forward_setup(g, cams, n_cams, o, gws, gws_bytes, pws, pws_bytes, n_entries, image, saved, f, true);
  if (rc) return rc;
  f.ra.penalty = penalty;
  hipStream_t s = (hipStream_t)stream;
  rc = build_lists(g, f.w, f.p, n_cams, f.ra.tiles_x, f.ra.tiles_y, o->full_coverage, f.cap, f.n_dev, s);
  if (rc) return rc;
  hipError_t e;
  {
    StageTimer t(S_RENDER_FWD, s);
    e = launch_render_forward(f.ra, f.cs, o->n_moments, o->n_intervals, s, o->basis == 1 ? kModeTrig : kModePlain);
  }
  if (e != hipSuccess) return hip_fail(e, "render_forward");
  return MB_OK;
}

int mb_render_forward_harvest(const mb_gaussians* g, const mb_camera* cams, int32_t n_cams, const mb_options* o,
                              void* gws, size_t gws_bytes, void* pws, size_t pws_bytes, int64_t n_entries,
                              float rate, uint32_t seed, float* samples, int32_t capacity, int32_t* count,
                              float* image, float* saved, void* stream) {
  FwdSetup f;
  int rc = forward_setup(g, cams, n_cams, o, gws, gws_bytes, pws, pws_bytes, n_entries, image, saved, f);
  if (rc) return rc;
  if (o->n_moments != 6) return fail(MB_ERR_ARG, "the surrogate's samples need n_moments = 6");
  if (!(rate >= 0.f && rate <= 1.f)) return fail(MB_ERR_ARG, "harvest rate must lie in [0, 1]");
  if (capacity < 0 || !count || (capacity > 0 && !samples)) return fail(MB_ERR_ARG, "bad sample buffer");
  hipStream_t s = (hipStream_t)stream;
  rc = build_lists(g, f.w, f.p, n_cams, f.ra.tiles_x, f.ra.tiles_y, o->full_coverage, n_entries, nullptr, s, false);
  if (rc) return rc;
  f.ra.harvest = samples;
  f.ra.harvest_count = count;
  f.ra.harvest_cap = capacity;
  f.ra.harvest_rate = rate;
  f.ra.seed = seed;
  hipError_t e;
  {
    StageTimer t(S_RENDER_FWD, s);
    e = launch_render_forward(f.ra, f.cs, o->n_moments, o->n_intervals, s, kModeHarvest);
  }
  if (e != hipSuccess) return hip_fail(e, "render_forward_harvest");
  return MB_OK;
}

size_t mb_query_workspace_bytes(int32_t n_cams, int32_t width, int32_t height, int64_t query_capacity) {
  if (n_cams < 1 || width <= 0 || height <= 0 || query_capacity < 0) return 0;
  return carve_queries(nullptr, (int64_t)n_cams * width * height, query_capacity).bytes;
}

size_t mb_query_workspace_bytes_backward(int32_t n_cams, int32_t width, int32_t height, int64_t query_capacity) {
  if (n_cams < 1 || width <= 0 || height <= 0 || query_capacity < 0) return 0;
  return carve_queries(nullptr, (int64_t)n_cams * width * height, query_capacity, true).bytes;
}

int mb_render_forward_surrogate(const mb_gaussians* g, const mb_camera* cams, int32_t n_cams, const mb_options* o,
                                void* gws, size_t gws_bytes, void* pws, size_t pws_bytes, int64_t n_entries,
                                const void* mlp_packed, void* qws, size_t qws_bytes, int64_t query_capacity,
                                float* image, float* saved, void* stream) {
  FwdSetup f;
  int rc = forward_setup(g, cams, n_cams, o, gws, gws_bytes, pws, pws_bytes, n_entries, image, saved, f);
  if (rc) return rc;
  if (o->n_moments != 6) return fail(MB_ERR_ARG, "the surrogate takes n_moments = 6");
  if (!mlp_packed) return fail(MB_ERR_ARG, "null surrogate weights");
  if (query_capacity < 0) return fail(MB_ERR_ARG, "negative query capacity");
  int64_t n_pix = (int64_t)n_cams * cams[0].width * cams[0].height;
  QueryWs q = carve_queries(qws, n_pix, query_capacity);
  if (!qws || qws_bytes < q.bytes)
    return fail(MB_ERR_WORKSPACE, "query workspace needs %zu bytes, got %zu", q.bytes, qws_bytes);
  hipStream_t s = (hipStream_t)stream;
  rc = build_lists(g, f.w, f.p, n_cams, f.ra.tiles_x, f.ra.tiles_y, o->full_coverage, n_entries, nullptr, s, false);
  if (rc) return rc;
  RenderArgs& ra = f.ra;
  ra.pixfeat = q.pixfeat;
  ra.pix_qbase = q.pix_qbase;
  ra.q_count = q.count;
  ra.q_cap = query_capacity;
  ra.q_z = q.q_z;
  ra.q_pix = q.q_pix;
  ra.q_f = q.q_f;
  hipError_t e = hipMemsetAsync(q.count, 0, sizeof(unsigned long long), s);
  if (e != hipSuccess) return hip_fail(e, "query counter reset");
  {
    StageTimer t(S_RENDER_FWD, s);
    e = launch_render_forward(ra, f.cs, o->n_moments, o->n_intervals, s, kModeEmit);
  }
  if (e != hipSuccess) return hip_fail(e, "render_forward (surrogate queries)");
  {
    StageTimer t(S_MLP, s);
    e = launch_mlp_forward_gather(mlp_packed, q.pixfeat, n_pix, q.q_pix, q.q_z, q.count, query_capacity, q.q_f, s);
  }
  if (e != hipSuccess) return hip_fail(e, "surrogate inference");
  {
    StageTimer t(S_CONSUME, s);
    e = launch_render_consume(ra, f.cs, o->n_intervals, s);
  }
  if (e != hipSuccess) return hip_fail(e, "render_forward (surrogate quadrature)");
  return MB_OK;
}

size_t mb_table_workspace_bytes(int32_t n_cams, int32_t width, int32_t height, int32_t n_nodes) {
  if (n_cams < 1 || width <= 0 || height <= 0 || n_nodes < 2 || n_nodes > kTabMaxNodes) return 0;
  const size_t n_pix = (size_t)n_cams * width * height;
  Carver c(nullptr);
  c.take<float>(n_pix * kPixFeat);
  c.take<float>(n_pix * (size_t)n_nodes);
  return c.off;
}

int mb_render_forward_tabulated(const mb_gaussians* g, const mb_camera* cams, int32_t n_cams, const mb_options* o,
                                void* gws, size_t gws_bytes, void* pws, size_t pws_bytes, int64_t n_entries,
                                const void* mlp_packed, int32_t n_nodes, void* tws, size_t tws_bytes, float* image,
                                float* saved, void* stream) {
  FwdSetup f;
  int rc = forward_setup(g, cams, n_cams, o, gws, gws_bytes, pws, pws_bytes, n_entries, image, saved, f);
  if (rc) return rc;
  if (o->basis != 0) return fail(MB_ERR_UNSUPPORTED, "the tabulated schedule takes power moments (basis 0)");
  if (mlp_packed && o->n_moments != 6) return fail(MB_ERR_ARG, "the surrogate takes n_moments = 6");
  if (!mlp_packed && o->n_moments == 8) return fail(MB_ERR_UNSUPPORTED, "tabulated bounds: n_moments 4 or 6");
  if (n_nodes < 2 || n_nodes > kTabMaxNodes) return fail(MB_ERR_ARG, "n_nodes must lie in [2, %d]", kTabMaxNodes);
  const int64_t n_pix = (int64_t)n_cams * cams[0].width * cams[0].height;
  const size_t need = mb_table_workspace_bytes(n_cams, cams[0].width, cams[0].height, n_nodes);
  if (!tws || tws_bytes < need) return fail(MB_ERR_WORKSPACE, "table workspace needs %zu bytes, got %zu", need, tws_bytes);
  Carver c(tws);
  float* pixfeat = c.take<float>((size_t)n_pix * kPixFeat);
  float* tab = c.take<float>((size_t)n_pix * n_nodes);
  hipStream_t s = (hipStream_t)stream;
  rc = build_lists(g, f.w, f.p, n_cams, f.ra.tiles_x, f.ra.tiles_y, o->full_coverage, n_entries, nullptr, s, false);
  if (rc) return rc;
  RenderArgs& ra = f.ra;
  ra.pixfeat = pixfeat;
  ra.tab = tab;
  ra.tab_nodes = n_nodes;
  hipError_t e;
  {
    StageTimer t(S_RENDER_FWD, s);
    e = launch_render_forward(ra, f.cs, o->n_moments, o->n_intervals, s, mlp_packed ? kModeTabSur : kModeTabPlain);
  }
  if (e != hipSuccess) return hip_fail(e, "render_forward (tabulated schedule)");
  if (mlp_packed) {
    StageTimer t(S_MLP, s);
    e = launch_mlp_table(mlp_packed, pixfeat, n_pix, n_nodes, tab, s);
    if (e != hipSuccess) return hip_fail(e, "surrogate table");
  }
  {
    StageTimer t(S_CONSUME, s);
    e = launch_render_consume_tab(ra, f.cs, o->n_intervals, s);
  }
  if (e != hipSuccess) return hip_fail(e, "render_forward (tabulated quadrature)");
  return MB_OK;
}

namespace {

// shared by the two backward entry points: checks, the render adjoint
// (plain, or through the surrogate's query list when q is given), and the
// per-Gaussian gradient reduction
int backward_common(const mb_gaussians* g, const mb_camera* cams, int32_t n_cams, const mb_options* o, void* gws,
                    size_t gws_bytes, void* pws, size_t pws_bytes, int64_t n_entries, const float* saved,
                    const float* grad_image, const float* grad_penalty, float* g_means, float* g_scales,
                    float* g_quats, float* g_densities, float* g_colors, hipStream_t s, const void* mlp_packed,
                    const QueryWs* q, int64_t query_capacity) {
  int tx = tiles_of(cams[0].width), ty = tiles_of(cams[0].height);
  int n_keys = tx * ty * n_cams;
  GaussWs w = carve_gauss(gws, g->n, n_cams);
  if (!gws || gws_bytes < w.bytes)
    return fail(MB_ERR_WORKSPACE, "Gaussian workspace needs %zu bytes, got %zu", w.bytes, gws_bytes);
  if (n_entries == MB_ENTRIES_ON_DEVICE) {  // the layout the forward used with this workspace
    n_entries = pws ? pair_capacity(pws_bytes, n_cams, cams[0].width, cams[0].height) : -1;
    if (n_entries < 0) return fail(MB_ERR_WORKSPACE, "pair workspace of %zu bytes holds no list", pws_bytes);
  }
  PairWs p = carve_pairs(pws, n_entries, n_keys, (int64_t)n_cams * cams[0].width * cams[0].height);
  if (!pws || pws_bytes < p.bytes)
    return fail(MB_ERR_WORKSPACE, "pair workspace needs %zu bytes, got %zu", p.bytes, pws_bytes);
  CamSet cs = make_cams(cams, n_cams);
  RenderArgs ra;
  memset(&ra, 0, sizeof(ra));
  ra.rec = w.rec; ra.sorted_rec = p.sorted_rec; ra.ranges = p.ranges; ra.order = p.order;
  ra.masks = p.masks;
  ra.pix_mom = p.pix_mom;
  ra.n_pix = (long long)n_cams * cams[0].width * cams[0].height;
  ra.tiles_x = tx; ra.tiles_y = ty; ra.n_cams = n_cams; ra.full_coverage = o->full_coverage;
  ra.kappa = o->kappa; ra.beta = o->beta; ra.eps = o->eps;
  fill_quantiles(o, ra.xq, ra.eq, ra.ecq);
  hipError_t e;
  if (q) {
    int64_t n_pix = (int64_t)n_cams * cams[0].width * cams[0].height;
    {
      StageTimer t(S_MLP, s);
      e = launch_mlp_input_grad_gather(mlp_packed, q->pixfeat, n_pix, q->q_pix, q->q_z, q->count, query_capacity,
                                       q->q_g, s);
    }
    if (e != hipSuccess) return hip_fail(e, "surrogate input gradients");
    ra.pixfeat = q->pixfeat;
    ra.pix_qbase = q->pix_qbase;
    ra.q_count = q->count;
    ra.q_cap = query_capacity;
    ra.q_f = q->q_f;
    ra.q_g = q->q_g;
  }
  {
    StageTimer t(S_RENDER_BWD, s);
    // 0: power moments, 1: the surrogate, 2: trigonometric moments
    const int mode = q != nullptr ? 1 : (o->basis == 1 ? 2 : 0);
    e = launch_render_backward(ra, saved, grad_image, grad_penalty, p.vals_a, p.partials, p.used, cs,
                               o->n_moments, o->n_intervals, s, mode);
  }
  if (e != hipSuccess) return hip_fail(e, "render_backward");
  GradArgs ga;
  ga.means = g->means; ga.scales = g->scales; ga.quats = g->quats; ga.dens = g->densities; ga.colors = g->colors;
  ga.n = g->n; ga.sh_degree = g->sh_degree;
  ga.counts = w.counts; ga.offsets = w.offsets; ga.partials = p.partials; ga.used = p.used;
  ga.e_cap = n_entries;
  ga.g_means = g_means; ga.g_scales = g_scales; ga.g_quats = g_quats; ga.g_dens = g_densities;
  ga.g_colors = g_colors;
  {
    StageTimer t(S_GRADS, s);
    e = launch_grad_finalize(ga, cs, s);
  }
  if (e != hipSuccess) return hip_fail(e, "gradients");
  return MB_OK;
}

int check_backward_args(const mb_gaussians* g, const mb_camera* cams, int32_t n_cams, const mb_options* o,
                        int64_t n_entries, const float* saved, const float* grad_image, float* g_means,
                        float* g_scales, float* g_quats, float* g_densities, float* g_colors,
                        bool device_count_ok = false) {
  int rc = check_common(g, cams, n_cams, o);
  if (rc) return rc;
  if (!saved || !grad_image) return fail(MB_ERR_ARG, "null saved state or image gradient");
  if (g->n > 0 && (!g_means || !g_scales || !g_quats || !g_densities || !g_colors))
    return fail(MB_ERR_ARG, "null gradient output");
  if (n_entries < 0 && !(device_count_ok && n_entries == MB_ENTRIES_ON_DEVICE))
    return fail(MB_ERR_ARG, "n_entries %lld is neither a count nor accepted here as MB_ENTRIES_ON_DEVICE",
                (long long)n_entries);
  return MB_OK;
}

}  // namespace

int mb_render_backward(const mb_gaussians* g, const mb_camera* cams, int32_t n_cams, const mb_options* o, void* gws,
                       size_t gws_bytes, void* pws, size_t pws_bytes, int64_t n_entries, const float* saved,
                       const float* grad_image, const float* grad_penalty, float* g_means, float* g_scales,
                       float* g_quats, float* g_densities, float* g_colors, void* stream) {
  int rc = check_backward_args(g, cams, n_cams, o, n_entries, saved, grad_image, g_means, g_scales, g_quats,
                               g_densities, g_colors, true);
  if (rc) return rc;
  return backward_common(g, cams, n_cams, o, gws, gws_bytes, pws, pws_bytes, n_entries, saved, grad_image,
                         grad_penalty, g_means, g_scales, g_quats, g_densities, g_colors, (hipStream_t)stream,
                         nullptr, nullptr, 0);
}

int mb_render_backward_surrogate(const mb_gaussians* g, const mb_camera* cams, int32_t n_cams, const mb_options* o,
                                 void* gws, size_t gws_bytes, void* pws, size_t pws_bytes, int64_t n_entries,
                                 const void* mlp_packed, void* qws, size_t qws_bytes, int64_t query_capacity,
                                 const float* saved, const float* grad_image, float* g_means, float* g_scales,
                                 float* g_quats, float* g_densities, float* g_colors, void* stream) {
  int rc = check_backward_args(g, cams, n_cams, o, n_entries, saved, grad_image, g_means, g_scales, g_quats,
                               g_densities, g_colors);
  if (rc) return rc;
  if (o->n_moments != 6) return fail(MB_ERR_ARG, "the surrogate takes n_moments = 6");
  if (!mlp_packed) return fail(MB_ERR_ARG, "null surrogate weights");
  if (query_capacity < 0) return fail(MB_ERR_ARG, "negative query capacity");
  int64_t n_pix = (int64_t)n_cams * cams[0].width * cams[0].height;
  QueryWs q = carve_queries(qws, n_pix, query_capacity, true);
  if (!qws || qws_bytes < q.bytes)
    return fail(MB_ERR_WORKSPACE, "query workspace needs %zu bytes, got %zu", q.bytes, qws_bytes);
  return backward_common(g, cams, n_cams, o, gws, gws_bytes, pws, pws_bytes, n_entries, saved, grad_image,
                         nullptr, g_means, g_scales, g_quats, g_densities, g_colors, (hipStream_t)stream,
                         mlp_packed, &q, query_capacity);
}

// ---------------------------------------------------------------------------
// D-SSIM term of the training objective
// ---------------------------------------------------------------------------
size_t mb_l1_workspace_bytes(void) { return (size_t)l1_partials() * sizeof(double); }

int mb_l1(const float* image, const float* target, int64_t n, float grad_scale, float* loss, float* grad_image,
          void* ws, size_t ws_bytes, void* stream) {
  if (n < 0) return fail(MB_ERR_ARG, "negative count");
  if (!loss || (n > 0 && (!image || !target))) return fail(MB_ERR_ARG, "null image, target or loss");
  if (!ws || ws_bytes < mb_l1_workspace_bytes())
    return fail(MB_ERR_WORKSPACE, "L1 workspace needs %zu bytes, got %zu", mb_l1_workspace_bytes(), ws_bytes);
  hipError_t e = launch_l1(image, target, n, grad_scale, loss, grad_image, (double*)ws, (hipStream_t)stream);
  return e == hipSuccess ? MB_OK : hip_fail(e, "l1");
}

size_t mb_dssim_workspace_bytes(int32_t n_cams, int32_t width, int32_t height) {
  if (n_cams < 1 || width <= 0 || height <= 0) return 0;
  Carver c(nullptr);
  c.take<float>((size_t)n_cams * width * height * 9);
  c.take<float>((size_t)dssim_blocks(n_cams, width, height));
  return c.off;
}

int mb_dssim(const float* image, const float* target, int32_t n_cams, int32_t width, int32_t height,
             float grad_scale, float* loss, float* grad_image, void* ws, size_t ws_bytes, void* stream) {
  if (n_cams < 1 || width <= 0 || height <= 0 || width > 16384 || height > 16384)
    return fail(MB_ERR_ARG, "bad image size");
  if (!image || !target || !loss) return fail(MB_ERR_ARG, "null image, target or loss");
  size_t need = mb_dssim_workspace_bytes(n_cams, width, height);
  if (!ws || ws_bytes < need) return fail(MB_ERR_WORKSPACE, "D-SSIM workspace needs %zu bytes, got %zu", need, ws_bytes);
  Carver c(ws);
  SsimArgs a;
  a.image = image;
  a.target = target;
  a.n_cams = n_cams;
  a.w = width;
  a.h = height;
  double gs[11], sum = 0.0;
  for (int k = 0; k < 11; ++k) {
    const double x = k - 5;
    gs[k] = std::exp(-x * x / (2.0 * 1.5 * 1.5));
    sum += gs[k];
  }
  for (int k = 0; k < 11; ++k) a.g[k] = (float)(gs[k] / sum);
  float* coef = c.take<float>((size_t)n_cams * width * height * 9);
  a.coef = grad_image ? coef : nullptr;
  a.partials = c.take<float>((size_t)dssim_blocks(n_cams, width, height));
  a.loss = loss;
  a.grad = grad_image;
  a.grad_scale = grad_scale;
  hipError_t e = launch_dssim(a, (hipStream_t)stream);
  return e == hipSuccess ? MB_OK : hip_fail(e, "dssim");
}

// ---------------------------------------------------------------------------
// Adaptive density control (App. E)
// ---------------------------------------------------------------------------
namespace {
int check_gaussians(const mb_gaussians* g) {
  if (!g) return fail(MB_ERR_ARG, "null gaussians");
  if (g->n < 0) return fail(MB_ERR_ARG, "negative Gaussian count %d", g->n);
  if (g->n > 0 && (!g->means || !g->scales || !g->quats || !g->densities || !g->colors))
    return fail(MB_ERR_ARG, "null Gaussian parameter pointer");
  if (g->sh_degree < -1 || g->sh_degree > 3) return fail(MB_ERR_UNSUPPORTED, "SH degree %d not in -1..3", g->sh_degree);
  return MB_OK;
}
}  // namespace

int mb_view_independent_opacity(const mb_gaussians* g, float* opacity, void* stream) {
  int rc = check_gaussians(g);
  if (rc) return rc;
  if (g->n > 0 && !opacity) return fail(MB_ERR_ARG, "null opacity output");
  hipError_t e = launch_vi_opacity(g->n, g->scales, g->densities, opacity, (hipStream_t)stream);
  return e == hipSuccess ? MB_OK : hip_fail(e, "view_independent_opacity");
}

int mb_density_from_opacity(int32_t n, const float* opacity, const float* scales, float* densities, void* stream) {
  if (n < 0) return fail(MB_ERR_ARG, "negative count");
  if (n > 0 && (!opacity || !scales || !densities)) return fail(MB_ERR_ARG, "null argument");
  hipError_t e = launch_density_from_opacity(n, opacity, scales, densities, (hipStream_t)stream);
  return e == hipSuccess ? MB_OK : hip_fail(e, "density_from_opacity");
}

int mb_adc_accumulate(int32_t n, const float* g_means, float* grad_acc, int32_t* grad_count, void* stream) {
  if (n < 0) return fail(MB_ERR_ARG, "negative count");
  if (n > 0 && (!g_means || !grad_acc || !grad_count)) return fail(MB_ERR_ARG, "null argument");
  hipError_t e = launch_adc_accumulate(n, g_means, grad_acc, grad_count, (hipStream_t)stream);
  return e == hipSuccess ? MB_OK : hip_fail(e, "adc_accumulate");
}

size_t mb_adc_workspace_bytes(int32_t n) {
  if (n < 0) return 0;
  Carver c(nullptr);
  c.take<int>((size_t)n);                 // output counts
  c.take<int>(scan_tmp_ints(n));
  return c.off;
}

int mb_adc_plan(const mb_gaussians* g, const float* grad_acc, const int32_t* grad_count, const mb_adc_params* p,
                int32_t* action, int32_t* offsets, int32_t* n_out, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_gaussians(g);
  if (rc) return rc;
  if (!p || !n_out) return fail(MB_ERR_ARG, "null parameters or count output");
  if (g->n > 0 && (!grad_acc || !grad_count || !action || !offsets)) return fail(MB_ERR_ARG, "null argument");
  size_t need = mb_adc_workspace_bytes(g->n);
  if (!ws || ws_bytes < need) return fail(MB_ERR_WORKSPACE, "ADC workspace needs %zu bytes, got %zu", need, ws_bytes);
  if ((int64_t)g->n * 2 >= (1ll << 31)) return fail(MB_ERR_ARG, "too many Gaussians");
  Carver c(ws);
  int* outs = c.take<int>((size_t)g->n);
  int* tmp = c.take<int>(scan_tmp_ints(g->n));
  AdcParams ap{p->min_opacity, p->grad_threshold, p->split_scale};
  hipError_t e = launch_adc_plan(g->n, g->scales, g->densities, grad_acc, grad_count, ap, action, outs, offsets, tmp,
                                 n_out, (hipStream_t)stream);
  return e == hipSuccess ? MB_OK : hip_fail(e, "adc_plan");
}

int mb_adc_apply(const mb_gaussians* g, const int32_t* action, const int32_t* offsets, float* means, float* scales,
                 float* quats, float* densities, float* colors, void* stream) {
  int rc = check_gaussians(g);
  if (rc) return rc;
  if (g->n > 0 && (!action || !offsets || !means || !scales || !quats || !densities || !colors))
    return fail(MB_ERR_ARG, "null argument");
  AdcApplyArgs a;
  a.n = g->n;
  a.color_stride = g->sh_degree < 0 ? 3 : 3 * (g->sh_degree + 1) * (g->sh_degree + 1);
  a.means = g->means; a.scales = g->scales; a.quats = g->quats; a.dens = g->densities; a.colors = g->colors;
  a.action = action; a.offsets = offsets;
  a.out_means = means; a.out_scales = scales; a.out_quats = quats; a.out_dens = densities; a.out_colors = colors;
  hipError_t e = launch_adc_apply(a, (hipStream_t)stream);
  return e == hipSuccess ? MB_OK : hip_fail(e, "adc_apply");
}

// ---------------------------------------------------------------------------
// Learned surrogate of the reconstruction (MLP, bf16 weights, fp32 accumulation)
// ---------------------------------------------------------------------------
int32_t mb_mlp_param_count(void) { return mlp_param_count(); }
size_t mb_mlp_packed_bytes(void) { return mlp_packed_bytes(); }
size_t mb_mlp_workspace_bytes(int64_t batch) { return batch < 0 ? 0 : mlp_workspace_bytes(batch); }

int mb_mlp_pack(const float* theta, void* packed, void* stream) {
  if (!theta || !packed) return fail(MB_ERR_ARG, "null parameter or packed-weight pointer");
  hipError_t e;
  {
    StageTimer t(S_MLP, (hipStream_t)stream);
    e = launch_mlp_pack(theta, packed, (hipStream_t)stream);
  }
  return e == hipSuccess ? MB_OK : hip_fail(e, "mlp_pack");
}

int mb_mlp_forward(const void* packed, const float* x, int64_t n, float* f_out, void* stream) {
  if (n < 0) return fail(MB_ERR_ARG, "negative batch");
  if (n > 0 && (!packed || !x || !f_out)) return fail(MB_ERR_ARG, "null MLP argument");
  hipError_t e;
  {
    StageTimer t(S_MLP, (hipStream_t)stream);
    e = launch_mlp_forward(packed, x, n, f_out, (hipStream_t)stream);
  }
  return e == hipSuccess ? MB_OK : hip_fail(e, "mlp_forward");
}

int mb_mlp_loss_grad(const void* packed, const float* x, const float* t_target, int64_t n, float* grad, float* loss,
                     void* ws, size_t ws_bytes, void* stream) {
  if (n <= 0) return fail(MB_ERR_ARG, "batch must be positive");
  if (!packed || !x || !t_target || !grad) return fail(MB_ERR_ARG, "null MLP argument");
  size_t need = mlp_workspace_bytes(n);
  if (!ws || ws_bytes < need) return fail(MB_ERR_WORKSPACE, "MLP workspace needs %zu bytes, got %zu", need, ws_bytes);
  hipError_t e;
  {
    StageTimer t(S_MLP, (hipStream_t)stream);
    e = launch_mlp_loss_grad(packed, x, t_target, n, grad, loss, (float*)ws, (hipStream_t)stream);
  }
  return e == hipSuccess ? MB_OK : hip_fail(e, "mlp_loss_grad");
}

int mb_adam_step(float* theta, float* m, float* v, const float* grad, int64_t count, int32_t step, float lr,
                 float beta1, float beta2, float eps, void* stream) {
  if (count <= 0 || !theta || !m || !v || !grad) return fail(MB_ERR_ARG, "bad Adam arguments");
  if (step < 1) return fail(MB_ERR_ARG, "Adam step counts from 1");
  hipError_t e;
  {
    StageTimer t(S_MLP, (hipStream_t)stream);
    e = launch_adam(theta, m, v, grad, count, step, lr, beta1, beta2, eps, (hipStream_t)stream);
  }
  return e == hipSuccess ? MB_OK : hip_fail(e, "adam");
}

int mb_render_forward_noalloc(const mb_gaussians* g, const mb_camera* cams, int32_t n_cams, const mb_options* o,
                              float* image, float* saved, float* penalty, int64_t* n_entries, void* stream) {
  int rc = check_common(g, cams, n_cams, o);
  if (rc) return rc;
  void* base = nullptr;
  rc = scratch_address(&base);
  if (rc) return rc;
  const size_t gws_bytes = (mb_gauss_workspace_bytes(g->n, n_cams) + 255) & ~size_t(255);
  if (gws_bytes > kScratchBytes)
    return fail(MB_ERR_WORKSPACE, "%d Gaussians x %d cameras need %zu bytes of Gaussian workspace; the "
                "allocation-free scratch holds %zu bytes", g->n, n_cams, gws_bytes, kScratchBytes);
  int64_t count = 0;
  rc = mb_prepare(g, cams, n_cams, o, base, gws_bytes, &count, stream);
  if (rc) return rc;
  const size_t pws_bytes = mb_pair_workspace_bytes(count, n_cams, cams[0].width, cams[0].height);
  if (pws_bytes == 0 || gws_bytes + pws_bytes > kScratchBytes)
    return fail(MB_ERR_WORKSPACE, "the frame's %lld tile entries need %zu + %zu bytes of workspace; the "
                "allocation-free scratch holds %zu bytes", (long long)count, gws_bytes, pws_bytes, kScratchBytes);
  if (n_entries) *n_entries = count;
  return mb_render_forward(g, cams, n_cams, o, base, gws_bytes, (unsigned char*)base + gws_bytes, pws_bytes,
                           count, image, saved, penalty, stream);
}

}  // extern "C"
