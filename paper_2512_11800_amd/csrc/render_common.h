// Per-pair building blocks shared by the forward and backward render
// kernels: LDS staging of render records, the coverage test, the ray-space
// Gaussian, the warped moments and the per-Gaussian quadrature.
#pragma once
#include "kernels.h"
#include "recon.h"

namespace mb {

struct Stage {
  float4 f[kRecF4][kBlock];
};

struct RayG {
  float mu, sig, omega;
  float id, xid, ek;  // 1 / D, X / D and exp(-X / 2D) at the pixel offset (for the adjoint)
};

// ---------------------------------------------------------------------------
// Per-wave compaction of covering pairs. A wave owns an 8x8 pixel block; while
// it walks the staged list, the (entry, pixel) pairs that pass the coverage
// test are appended to a queue in (entry, pixel) order and evaluated 64 at a
// time, one pair per lane, so the arithmetic runs on full waves whatever the
// fraction of the block a Gaussian covers. A pair's results go back to the
// pixel's own lane (the owner), which adds them in queue order: per pixel the
// summation order is the list order, as without compaction.
// ---------------------------------------------------------------------------
struct WaveQueue {
  uint16_t item[128];  // (entry in the staged batch) << 6 | pixel lane
};

// Optional rank tracking beside a queue: q[pos] receives the pair's index
// among its pixel's covering pairs, counted by the pixel lane's ctr. Kept out
// of WaveQueue so the kernels that do not need it spend no LDS on it.
struct QueueRanks {
  uint32_t* q;  // [128] in LDS, parallel to WaveQueue::item
  uint32_t ctr;
};

struct QueueCursor {
  int cnt;                  // queued pairs (wave-uniform)
  uint64_t own_lo, own_hi;  // this lane's queue positions [0, 64) and [64, 128)
};

__device__ __forceinline__ void queue_reset(QueueCursor& qc) {
  qc.cnt = 0;
  qc.own_lo = 0;
  qc.own_hi = 0;
}

// Append this lane's pair (entry j) if cov; all lanes call it with the same
// ballot mask. Returns the new count.
__device__ __forceinline__ void queue_push(WaveQueue& q, QueueCursor& qc, uint64_t mask, bool cov, int j,
                                           int lane, QueueRanks* rank = nullptr) {
  if (cov) {
    int pos = qc.cnt + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
    q.item[pos] = (uint16_t)((j << 6) | lane);
    if (rank) rank->q[pos] = rank->ctr++;
    if (pos < 64)
      qc.own_lo |= 1ull << pos;
    else
      qc.own_hi |= 1ull << (pos - 64);
  }
  qc.cnt += __popcll(mask);
}

// After evaluating positions [0, 64): move the rest to the front (with their
// ranks when RANK: only a queue filled with ranks needs them).
template <bool RANK = false>
__device__ __forceinline__ void queue_pop64(WaveQueue& q, QueueCursor& qc, int lane, uint32_t* rq = nullptr) {
  int rest = qc.cnt - 64;
  uint16_t it = lane < rest ? q.item[64 + lane] : (uint16_t)0;
  uint32_t rk = (RANK && lane < rest) ? rq[64 + lane] : 0u;
  __builtin_amdgcn_wave_barrier();
  if (lane < rest) {
    q.item[lane] = it;
    if (RANK) rq[lane] = rk;
  }
  __builtin_amdgcn_wave_barrier();
  qc.own_lo = qc.own_hi;
  qc.own_hi = 0;
  qc.cnt = rest;
}

// Queue the pairs of the staged batch [b, b + nb) from the stored coverage
// masks of this wave (restricted to the lanes of `keep`), skipping empty
// entries 64 at a time. on_full() evaluates and pops 64 queued pairs;
// on_empty(j) is called by the lane that loaded entry j's mask when the
// stored mask has pixels but none of them is kept.
// In a split block (see BlockWork) a wave takes only the entries j with
// j % 4 == its wave index (`own4` >= 0); otherwise every entry (`own4` < 0).
// PREFETCH: the masks of the next 64 entries are loaded before the current
// 64 are queued and evaluated, so that their latency hides behind that work
// (two more registers live across the evaluation: the forward kernels gain,
// the register-bound backward does not).
template <bool PREFETCH = false, class Full, class Empty>
__device__ __forceinline__ void queue_from_masks(WaveQueue& q, QueueCursor& qc, const uint64_t* masks, int b, int nb,
                                                 int quad, int own4, int lane, uint64_t keep, Full&& on_full,
                                                 Empty&& on_empty, QueueRanks* rank = nullptr) {
  auto load = [&](int j0) __attribute__((always_inline)) {
    const bool in = j0 + lane < nb && (own4 < 0 || ((j0 + lane) & 3) == own4);
    return in ? masks[(size_t)(b + j0 + lane) * 4 + quad] : 0ull;
  };
  uint64_t next = PREFETCH ? load(0) : 0ull;
  for (int j0 = 0; j0 < nb; j0 += 64) {
    const bool in = j0 + lane < nb && (own4 < 0 || ((j0 + lane) & 3) == own4);
    uint64_t raw;
    if constexpr (PREFETCH) {
      raw = next;
      next = j0 + 64 < nb ? load(j0 + 64) : 0ull;
    } else {
      raw = load(j0);
    }
    const uint64_t mk = raw & keep;
    if (in && mk == 0 && raw != 0) on_empty(j0 + lane);
    uint64_t nz = __ballot(mk != 0);
    while (nz) {
      const int l = __builtin_ctzll(nz);
      nz &= nz - 1;
      const uint64_t m = __shfl(mk, l, 64);
      queue_push(q, qc, m, (m >> lane) & 1ull, j0 + l, lane, rank);
      if (qc.cnt >= 64) on_full();
    }
  }
}

// Owner accumulation: calls add(load(i)) for this lane's own queue positions
// i (bits of `own`) in increasing order, two positions per iteration with
// both loads issued before either value is consumed.
template <class Load, class Add>
__device__ __forceinline__ void for_each_own(uint64_t own, Load&& load, Add&& add) {
  while (own) {
    const int i0 = __builtin_ctzll(own);
    own &= own - 1;
    const bool two = own != 0;
    const int i1 = two ? __builtin_ctzll(own) : i0;
    own &= own - 1;
    const auto v0 = load(i0);
    const auto v1 = load(i1);
    add(v0);
    if (two) add(v1);
  }
}

// value of pixel lane p (all lanes must take part)
__device__ __forceinline__ float from_lane(float v, int p) { return __shfl(v, p, 64); }

// Work of a render block (see launch_tile_order): tile key (camera * tiles +
// tile; n_keys for an empty block) and, for a block of a split tile, the
// quadrant its four waves share (quad = -1: the whole tile, one quadrant per
// wave).
struct BlockWork {
  int key, quad;
};
__device__ __forceinline__ BlockWork block_work(const RenderArgs& a) {
  const int code = a.order[blockIdx.x];
  BlockWork w;
  if (code >= 0) {
    w.key = code;
    w.quad = -1;
  } else {
    const int v = -code - 1;
    w.key = v >> 2;
    w.quad = v & 3;
  }
  return w;
}

__device__ __forceinline__ void load_batch(Stage& st, const float4* rec, const int* sorted_rec, int b, int nb) {
  int tid = threadIdx.x;
  if (tid < nb) {
    const float4* src = rec + (size_t)sorted_rec[b + tid] * kRecStride;
#pragma unroll
    for (int k = 0; k < kRecF4; ++k) st.f[k][tid] = src[k];
  }
}

// load_batch for the passes that walk the stored coverage masks: an entry
// whose masks are empty for every quadrant the block renders is never
// evaluated, so its record is not fetched (its staging slot keeps stale
// data that nothing reads). quad >= 0: a split block's one quadrant; -1: the
// whole tile (any of the four masks).
__device__ __forceinline__ void load_batch_covered(Stage& st, const float4* rec, const int* sorted_rec,
                                                   const uint64_t* masks, int quad, int b, int nb) {
  int tid = threadIdx.x;
  if (tid < nb) {
    const uint64_t* mp = masks + (size_t)(b + tid) * 4;
    bool need;
    if (quad >= 0) {
      need = mp[quad] != 0ull;
    } else {
      const ulonglong2 m01 = reinterpret_cast<const ulonglong2*>(mp)[0];
      const ulonglong2 m23 = reinterpret_cast<const ulonglong2*>(mp)[1];
      need = (m01.x | m01.y | m23.x | m23.y) != 0ull;
    }
    if (need) {
      const float4* src = rec + (size_t)sorted_rec[b + tid] * kRecStride;
#pragma unroll
      for (int k = 0; k < kRecF4; ++k) st.f[k][tid] = src[k];
    }
  }
}

// Coverage of the pixel centres of a tile by staged entry j, in the
// rectangle's axis coordinates c1 = (p - C) . e1, c2 = (p - C) . e2 (C, e1,
// e2 = e1 rotated by +90 degrees, halves h1, h2 from the record; covered iff
// |c1| <= h1 and |c2| <= h2). cover_setup evaluates (c1, c2) once per entry at
// the tile's first pixel centre (x_t + 1/2, y_t + 1/2); the per-pixel test
// adds the pixel's offset (i, j) inside the tile, c1 + i e1x + j e1y and
// c2 - i e1y + j e1x, two fused multiply-adds each. The float test decides
// wherever its margin to an edge exceeds `band`, a bound on its rounding
// error: the record's centre offset, axis and halves are the double values
// rounded to float (relative 2^-24), and the set-up and per-pixel operations
// round relative 2^-24 each; summed, the error stays below
// 2^-24 (9 (|a_x| + |a_y|) + 2 (|o_x| + |o_y|) + 2 (h1 + h2) + 100) (a: the
// tile origin's offset from the rectangle's centre, o: the centre's offset
// from the projected mean), and the band 1e-6 (16 + |a_x| + |a_y| + |o_x| +
// |o_y| + h1 + h2) is about twice that. Near an edge the wave re-tests in
// double against rectd. Only the first pass tests coverage: every later pass,
// forward and backward, reads the masks it stores.
//
// The set-up lives in LDS the kernel already holds: (c1, c2) at the tile
// origin replace the staged record's centre offset (st.f[0][j].zw, which
// the first pass reads nowhere else and the later passes stage again), and
// the band shares a 32-bit word with the quadrant bits (cover_word: the band's
// four low mantissa bits carry them; clearing them lowers the band by a
// relative 2^-19 at most).
//
// cover_setup also returns the 8x8 quadrants of the tile the rectangle can
// reach (bit q for quadrant q = 2 row + column): those whose pixel-centre
// square overlaps the rectangle's axis-aligned box, and whose centre lies
// within h + 3.5 (|e1x| + |e1y|) of the rectangle along both of its axes
// (the separating-axis test of two rectangles); a margin beyond the
// rounding bound keeps the bits from ever missing a covered pixel.
__device__ __forceinline__ uint32_t cover_setup(Stage& st, int j, int xt, int yt) {
  const float4 f0 = st.f[0][j], f1 = st.f[1][j];
  const float ax = ((float)xt + 0.5f - f0.x) - f0.z;
  const float ay = ((float)yt + 0.5f - f0.y) - f0.w;
  const float a1 = ax * f1.x + ay * f1.y;
  const float a2 = ay * f1.x - ax * f1.y;
  const float band = 1e-6f * (16.f + fabsf(ax) + fabsf(ay) + fabsf(f0.z) + fabsf(f0.w) + f1.z + f1.w);
  st.f[0][j] = make_float4(f0.x, f0.y, a1, a2);
  const float cx = f0.x + f0.z, cy = f0.y + f0.w;
  const float eax = fabsf(f1.x), eay = fabsf(f1.y);
  const float mx = 0.01f + 1e-5f * fabsf(cx), my = 0.01f + 1e-5f * fabsf(cy);
  const float bx = eax * f1.z + eay * f1.w + mx, by = eay * f1.z + eax * f1.w + my;
  const float reach = 3.5f * (eax + eay) + band + 0.01f;
  uint32_t bits = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float lx = (float)(xt + (q & 1) * 8) + 0.5f, ly = (float)(yt + (q >> 1) * 8) + 0.5f;
    const bool box = cx + bx >= lx && cx - bx <= lx + 7.f && cy + by >= ly && cy - by <= ly + 7.f;
    const float qi = 8.f * (float)(q & 1) + 3.5f, qj = 8.f * (float)(q >> 1) + 3.5f;
    const float c1 = a1 + qi * f1.x + qj * f1.y;
    const float c2 = a2 - qi * f1.y + qj * f1.x;
    const bool sat = fabsf(c1) <= f1.z + reach && fabsf(c2) <= f1.w + reach;
    bits |= (box && sat) ? (1u << q) : 0u;
  }
  return (__float_as_uint(band) & ~15u) | bits;
}

__device__ __forceinline__ bool cover_reaches(uint32_t word, int quad) { return (word >> quad) & 1u; }
__device__ __forceinline__ float cover_band(uint32_t word) { return __uint_as_float(word & ~15u); }

// The per-pixel test of entry j (after cover_setup; `word` its set-up word)
// for the pixel at offset (fi, fj) from the tile's first pixel, centre (u, v).
__device__ __forceinline__ bool covers(const Stage& st, uint32_t word, const double2* rectd, const int* sorted_rec,
                                       int b, int j, float fi, float fj, float u, float v, bool inside) {
  const float4 f0 = st.f[0][j], f1 = st.f[1][j];
  const float c1 = fmaf(fj, f1.y, fmaf(fi, f1.x, f0.z));
  const float c2 = fmaf(fj, f1.x, fmaf(fi, -f1.y, f0.w));
  const float m = fminf(f1.z - fabsf(c1), f1.w - fabsf(c2));
  bool cov = inside && m >= 0.f;
  const bool amb = inside && fabsf(m) < cover_band(word);
  if (__ballot(amb) != 0) {
    const int rid = __builtin_amdgcn_readfirstlane(sorted_rec[b + j]);
    const double2 cd = rectd[(size_t)rid * 3], ed = rectd[(size_t)rid * 3 + 1], hd = rectd[(size_t)rid * 3 + 2];
    if (amb) {
      const double axd = (double)u - cd.x, ayd = (double)v - cd.y;
      const double c1d = axd * ed.x + ayd * ed.y;
      const double c2d = -axd * ed.y + ayd * ed.x;
      cov = fabs(c1d) <= hd.x && fabs(c2d) <= hd.y;
    }
  }
  return cov;
}

// Mask walk without a queue: calls body(j, m) for every entry j of the staged
// batch [b, b + nb) whose 64-bit coverage mask m for this wave's pixel block
// `quad` is not zero, in list order (wave-uniform j and m).
template <class Body>
__device__ __forceinline__ void for_each_masked(const uint64_t* masks, int b, int nb, int quad, int lane,
                                                Body&& body) {
  uint64_t next = lane < nb ? masks[(size_t)(b + lane) * 4 + quad] : 0ull;
  for (int j0 = 0; j0 < nb; j0 += 64) {
    const uint64_t mk = next;  // the next 64 masks load while these are walked
    next = j0 + 64 + lane < nb ? masks[(size_t)(b + j0 + 64 + lane) * 4 + quad] : 0ull;
    uint64_t nz = __ballot(mk != 0);
    while (nz) {
      const int l = __builtin_ctzll(nz);
      nz &= nz - 1;
      body(j0 + l, (uint64_t)__shfl(mk, l, 64));
    }
  }
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
  g.id = id;
  g.xid = x * id;
  g.ek = exp_neg_half(g.xid);
  g.mu = lam * e * id;
  g.sig = lam * fast_rsq(d);
  g.omega = w * g.ek;
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
  float e = __expf(-bn * bn);
  float s2 = g.sig * g.sig;
  m[0] = g.omega * g.sig * kSqrtHalfPi * erfc_fast(bn);
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

// The same moments with the recurrence in double (from the float ray
// Gaussian): each pair's moment vector is then, to double rounding, the exact
// moment vector of a Gaussian, so the pixel's Hankel matrix keeps its small
// pivots. Independent float rounding of the nine moments of K = 8 moves a
// pivot of 1e-5 (relative) by several percent, enough to shift the bounds.
template <int K>
__device__ __forceinline__ void particle_moments_d(const RayG& g, const PixelBasis& pb, float tn, double* m) {
  float mus = fmaxf(g.mu, tn);
  float ys = warp_y(pb, mus, mus - pb.tc);
  float yp = warp_dy(pb, mus);
  const double gg = (double)ys + (double)yp * (double)(g.mu - mus);
  float is = fast_rcp(g.sig);
  float bn = (tn - g.mu) * kInvSqrt2 * is;
  float e = __expf(-bn * bn);
  const double s2 = (double)g.sig * (double)g.sig;
  m[0] = (double)(g.omega * g.sig * kSqrtHalfPi * erfc_fast(bn));
  const double bnd = (double)yp * (double)g.omega * s2 * (double)e;
  m[1] = gg * m[0] + bnd;
  const double un = gg + (double)yp * (double)(tn - g.mu);
  double unp = un;
  const double v2 = (double)yp * (double)yp * s2;
#pragma unroll
  for (int k = 2; k <= K; ++k) {
    m[k] = gg * m[k - 1] + (double)(k - 1) * v2 * m[k - 2] + bnd * unp;
    unp *= un;
  }
}

// phi(x) = (1 - e^-x) / x from d = e^-x: the Taylor series up to x^4 for
// |x| < 1/16 (truncation below 2e-9 relative), the direct form beyond (where
// 1 - d > 0.06, so its rounding stays below 1e-6 relative)
constexpr float kPhiSeries = 0.0625f;
__device__ __forceinline__ float phi_fn(float x, float d) {
  float s = 1.f / 120.f;
  s = fmaf(s, -x, 1.f / 24.f);
  s = fmaf(s, -x, 1.f / 6.f);
  s = fmaf(s, -x, 0.5f);
  s = fmaf(s, -x, 1.f);
  return fabsf(x) < kPhiSeries ? s : (1.f - d) * fast_rcp(x);
}

// Interval edges of one Gaussian's quadrature (App. B sample spacing): edge
// offsets, the clamp to the near bound, the moment variable y at each edge
// and the particle density sigma_i there.
template <int NQ>
struct QEdges {
  float off[NQ], y[NQ], sj[NQ], tau[NQ];
  bool cl[NQ];
};

template <int NQ>
__device__ __forceinline__ void quad_edges(const RayG& g, const PixelBasis& pb, float tn, const RenderArgs& a,
                                           QEdges<NQ>& e) {
  float dtc = g.mu - pb.tc;
  // every edge left of the near bound is moved onto it: one density there
  const float rn = (tn - g.mu) * fast_rcp(g.sig);
  const float en = exp_neg_half(rn * rn);
#pragma unroll
  for (int j = 0; j < NQ; ++j) {
    e.off[j] = a.kappa * g.sig * a.xq[j];
    float t = g.mu + e.off[j];
    e.cl[j] = t < tn;
    float dt = e.cl[j] ? (tn - pb.tc) : (dtc + e.off[j]);
    t = e.cl[j] ? tn : t;
    e.y[j] = warp_y(pb, t, dt);
    e.sj[j] = g.omega * (e.cl[j] ? en : a.eq[j]);
  }
}

// Eq. 7 sum over the intervals, given the optical depth at every edge
template <int NQ>
__device__ __forceinline__ float quad_sum(const RayG& g, float tn, const QEdges<NQ>& e) {
  float q = 0.f;
  float T = __expf(-e.tau[0]);  // transmittance at edge j, carried along the edges
#pragma unroll
  for (int j = 0; j + 1 < NQ; ++j) {
    float delta = e.cl[j + 1] ? 0.f : (e.cl[j] ? (g.mu + e.off[j + 1] - tn) : (e.off[j + 1] - e.off[j]));
    const float x = e.tau[j + 1] - e.tau[j];
    const float d = __expf(-x);
    q += T * delta * phi_fn(x, d) * e.sj[j];
    T *= d;
  }
  return q;
}

// Consistency penalty of one Gaussian (App. E, regularisation): over each
// quadrature interval the reconstructed optical depth may not grow by less
// than the particle's own depth there, tau_ij = omega Sigma sqrt(pi/2)
// (erfc(b_j) - erfc(b_{j+1})), b = (t - mu) / (sqrt2 Sigma); for an edge left
// of the near bound b is taken at t_n, otherwise it is kappa x_j / sqrt2.
// P_i = sum_j max(0, tau_ij - (tau_{j+1} - tau_j))^2.
template <int NQ>
__device__ __forceinline__ float pair_penalty(const RayG& g, float tn, const QEdges<NQ>& e, const RenderArgs& a) {
  bool any_cl = false;
#pragma unroll
  for (int j = 0; j < NQ; ++j) any_cl = any_cl || e.cl[j];
  const float en = any_cl ? erfc_fast((tn - g.mu) * kInvSqrt2 * fast_rcp(g.sig)) : 0.f;
  const float cs = g.omega * g.sig * kSqrtHalfPi;
  float pen = 0.f;
#pragma unroll
  for (int j = 0; j + 1 < NQ; ++j) {
    const float e0 = e.cl[j] ? en : a.ecq[j];
    const float e1 = e.cl[j + 1] ? en : a.ecq[j + 1];
    const float r = fmaxf(cs * (e0 - e1) - (e.tau[j + 1] - e.tau[j]), 0.f);
    pen += r * r;
  }
  return pen;
}

// Quadrature of Eq. 7 for one Gaussian against the pixel's moment bounds.
template <int NH, int NQ>
__device__ __forceinline__ float particle_quadrature(const RayG& g, const PixelBasis& pb, const LInv<NH>& L,
                                                     float m0, float tn, const RenderArgs& a, QEdges<NQ>& e) {
  quad_edges<NQ>(g, pb, tn, a, e);
#pragma unroll
  for (int j = 0; j < NQ; ++j) e.tau[j] = m0 * bound_F<NH>(L, e.y[j], a.beta);
  return quad_sum<NQ>(g, tn, e);
}

}  // namespace mb
