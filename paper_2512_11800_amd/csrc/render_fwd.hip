// Forward render: one workgroup per 16x16 tile (one thread per pixel, each
// wave an 8x8 quadrant). The tile's Gaussian list is streamed through LDS in
// batches of 256 records, three times:
//   pass 0  the pixel's moment variable (mean and spread of its depth mass),
//   pass 1  warped power moments, Eqs. 10-12, summed in double (Moment pass),
//   setup   Cholesky of the Hankel matrix, kept as L^-1 (Sec. 3.2),
//   pass 2  per-Gaussian quadrature, Eq. 7 / App. B, against the bounds
//           (Quadrature pass), accumulating sum q_i (r, g, b, 1),
//   epilogue  Eq. 15 rescaling (Rescale pass).
// Pass 0 tests coverage and stores, per list entry and wave, the 64-bit mask
// of covered pixels; the later passes (and the backward kernel) walk the
// masks instead. Covering pairs are evaluated compacted (see WaveQueue).
//
// Variants (MODE):
//   kModePlain    the path above;
//   kModeHarvest  the same, also writing a seeded pseudo-random subset of its
//                 queries as training samples of the learned surrogate
//                 (features, query, m_0 and the transmittance of the bounds);
//   kModeEmit     passes 0-1, then the surrogate's query list in place of the
//                 bound evaluation; k_render_consume completes the quadrature
//                 from the surrogate's outputs.
#include "render_common.h"
#include "trig.h"

namespace mb {

// Surrogate features of a pixel: the moments of its normalised measure in
// standardised form (mean 0, variance 1 in the moment variable), passed
// through asinh, and the map (y - mu) / sig of the moment variable onto the
// standardised one. The moment bounds are covariant under increasing affine
// maps of the variable, so F at a query depends on these alone.
__device__ __forceinline__ void surrogate_features(const double* acc, float* feat, float& mu, float& sig) {
  double b[7];
  b[0] = 1.0;
#pragma unroll
  for (int k = 1; k <= 6; ++k) b[k] = acc[k] / acc[0];
  const double m = b[1];
  const double var = b[2] - m * m;
  const double s = var > 0.0 ? sqrt(var) : 1.0;
  const double is = 1.0 / s;
  double c[7];  // central moments E[(y - m)^k]
  c[0] = 1.0;
#pragma unroll
  for (int k = 1; k <= 6; ++k) {
    // sum_j C(k, j) b_j (-m)^(k - j), with binomials built by the recurrence
    double acc_k = 0.0, binom = 1.0, pw = 1.0;
#pragma unroll
    for (int j = k; j >= 0; --j) {
      acc_k += binom * b[j] * pw;
      binom = binom * (double)j / (double)(k - j + 1);
      pw *= -m;
    }
    c[k] = acc_k;
  }
  double sk = 1.0;
#pragma unroll
  for (int k = 1; k <= 6; ++k) {
    sk *= is;
    feat[k - 1] = (float)asinh(c[k] * sk);
  }
  mu = (float)m;
  sig = (float)s;
}

// 32-bit integer hash for the harvest's sample selection
__device__ __forceinline__ uint32_t mix_hash(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u ^ (c + 0x165667B1u) * 0xC2B2AE3Du;
  h ^= h >> 16;
  h *= 0x7FEB352Du;
  h ^= h >> 15;
  h *= 0x846CA68Bu;
  h ^= h >> 16;
  return h;
}

constexpr float kMaxZ = 10.f;  // clamp of the standardised query

__device__ __forceinline__ float std_query(float y, float mu, float sig) {
  return fminf(fmaxf((y - mu) / sig, -kMaxZ), kMaxZ);
}

template <int K, int NQ, int MODE>
__global__ __launch_bounds__(256) void k_render_fwd(RenderArgs a, CamSet cams) {
  constexpr int NH = K / 2;
  __shared__ Stage st;
  __shared__ long long s_base;
  __shared__ int s_scan[4];
  const int tiles_per_cam = a.tiles_x * a.tiles_y;
  const int n_keys = tiles_per_cam * a.n_cams;
  const BlockWork bw = block_work(a);
  const int key = bw.key;
  if (key >= n_keys) return;
  const int ci = key / tiles_per_cam;
  const int tile = key - ci * tiles_per_cam;
  const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
  const CamConst& c = cams.c[ci];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // the wave's 8x8 pixel block; in a split block all four waves share one
  // and each takes every fourth list entry (own4)
  const bool split = bw.quad >= 0;
  const int quad = split ? bw.quad : wave;
  const int own4 = split ? wave : -1;
  const int px = tx * kTile + (quad & 1) * 8 + (lane & 7);
  const int py = ty * kTile + (quad >> 1) * 8 + (lane >> 3);
  const bool inside = px < c.width && py < c.height;
  const float u = (float)px + 0.5f, v = (float)py + 0.5f;
  const float fi = (float)(px - tx * kTile), fj = (float)(py - ty * kTile);  // offset inside the tile
  const float rx = (u - c.cx) / c.fx, ry = (v - c.cy) / c.fy;
  const float lam = sqrtf(1.f + rx * rx + ry * ry);
  const float tn = c.tn;
  const int2 rg = a.ranges[key];
  const size_t pix = ((size_t)ci * c.height + (inside ? py : 0)) * c.width + (inside ? px : 0);

  __shared__ WaveQueue wq[4];
  __shared__ uint32_t reach[kBlock];  // per staged entry: its coverage set-up word (cover_setup)
  // per-wave results of the queued pairs: 3 or K + 1 floats per pair in passes
  // 0 and 1, q (r, g, b, 1) in pass 2
  // (K = 8 and the trigonometric moments pass their moments in double:
  // twice the room)
  constexpr bool kTrig = MODE == kModeTrig;
  constexpr bool kDblMom = K >= 8 || kTrig;
  __shared__ __align__(16) float wres[4][(K + 1) * 64 * (kDblMom ? 2 : 1)];
  WaveQueue& q = wq[wave];
  float* res = wres[wave];
  const int x0 = tx * kTile + (quad & 1) * 8, y0 = ty * kTile + (quad >> 1) * 8;
  // partial per-pixel sums of a split block's four waves, combined in wave
  // order through the (then idle) staging buffer; every wave ends with the
  // same totals
  float* xch = reinterpret_cast<float*>(&st);
  // the pair at queue position `lane` (entry j, pixel lane p); inactive lanes
  // (lane >= n) get p = lane so the cross-lane reads stay uniform
  auto item_of = [&](int n, int& j, int& p) __attribute__((always_inline)) {
    const bool act = lane < n;
    const int it = act ? (int)q.item[lane] : lane;
    j = act ? (it >> 6) : 0;
    p = it & 63;
    return act;
  };
  auto ray_of = [&](int j, int p, float lamp) __attribute__((always_inline)) {
    const float dx = (float)(x0 + (p & 7)) + 0.5f - st.f[0][j].x;
    const float dy = (float)(y0 + (p >> 3)) + 0.5f - st.f[0][j].y;
    return ray_params(st, j, dx, dy, lamp);
  };

  // ---- pass 0: coverage masks and the pixel's moment variable --------------
  // weighted depth statistics of the covering Gaussians (weight omega Sigma):
  // sums of w, w mu and w (mu^2 + Sigma^2) in double (weights can be denormal
  // floats; the variance is a difference of these sums)
  double sw = 0.0, swm = 0.0, swq = 0.0;
  int n_cov = 0;
  {
    auto flush = [&](int n, uint64_t own) __attribute__((always_inline)) {
      int j, p;
      const bool act = item_of(n, j, p);
      const float lamp = from_lane(lam, p);
      if (act) {
        RayG g = ray_of(j, p, lamp);
        res[lane] = g.omega * g.sig;
        res[64 + lane] = g.mu;
        res[128 + lane] = g.sig;
      }
      __builtin_amdgcn_wave_barrier();
      while (own) {
        const int i = __builtin_ctzll(own);
        own &= own - 1;
        const double wgt = (double)res[i], mu = (double)res[64 + i], sg = (double)res[128 + i];
        sw += wgt;
        swm = fma(wgt, mu, swm);
        swq = fma(wgt, fma(mu, mu, sg * sg), swq);
      }
      __builtin_amdgcn_wave_barrier();
    };
    for (int b = rg.x; b < rg.y; b += kBlock) {
      int nb = min(kBlock, rg.y - b);
      __syncthreads();
      load_batch(st, a.rec, a.sorted_rec, b, nb);
      // each thread reads back the record it staged itself
      if (tid < nb) reach[tid] = cover_setup(st, tid, tx * kTile, ty * kTile);
      __syncthreads();
      QueueCursor qc;
      queue_reset(qc);
      // entries whose rectangle's box misses this wave's 8x8 block cover none
      // of its pixels: their mask is zero and the per-pixel test is skipped;
      // the others are tested in list order
      for (int j0 = 0; j0 < nb; j0 += 64) {
        const int jl = j0 + lane;
        const bool mine = jl < nb && (own4 < 0 || (jl & 3) == own4);
        const bool near = mine && cover_reaches(reach[mine ? jl : 0], quad);
        if (mine && !near) a.masks[(size_t)(b + jl) * 4 + quad] = 0ull;
        uint64_t todo = __ballot(near);
        while (todo) {
          const int j = j0 + __builtin_ctzll(todo);
          todo &= todo - 1;
          const bool cov = covers(st, reach[j], a.rectd, a.sorted_rec, b, j, fi, fj, u, v, inside);
          uint64_t mask = __ballot(cov);
          if (lane == 0) a.masks[(size_t)(b + j) * 4 + quad] = mask;
          if (mask == 0) continue;
          n_cov += cov ? 1 : 0;
          queue_push(q, qc, mask, cov, j, lane);
          if (qc.cnt >= 64) {
            flush(64, qc.own_lo);
            queue_pop64(q, qc, lane);
          }
        }
      }
      if (qc.cnt > 0) flush(qc.cnt, qc.own_lo);
    }
  }
  if (split) {
    // add the four waves' sums in wave order
    double* xd = reinterpret_cast<double*>(&st);
    __syncthreads();
    xd[(wave * 4 + 0) * 64 + lane] = sw;
    xd[(wave * 4 + 1) * 64 + lane] = swm;
    xd[(wave * 4 + 2) * 64 + lane] = swq;
    xd[(wave * 4 + 3) * 64 + lane] = (double)n_cov;
    __syncthreads();
    sw = swm = swq = 0.0;
    n_cov = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      sw += xd[(w * 4 + 0) * 64 + lane];
      swm += xd[(w * 4 + 1) * 64 + lane];
      swq += xd[(w * 4 + 2) * 64 + lane];
      n_cov += (int)xd[(w * 4 + 3) * 64 + lane];
    }
  }
  float mean = 0.f, var = 0.f;
  if (sw > 0.0) {
    const double md = swm / sw;
    mean = (float)md;
    var = (float)fmax(swq / sw - md * md, 0.0);
  }
  float tc = fmaxf(mean, tn);
  float sd = var > 0.f ? sqrtf(var) : 1.f;
  {
    float qq = 1.f + 0.8f * tc, xn = 1.f + 0.8f * tn;
    float gp = 1.2f * xn * sqrtf(xn) / (qq * qq * sqrtf(qq));  // g_hat'(tc)
    sd = fmaxf(sd * gp, 1e-30f);
  }
  const PixelBasis pb = make_basis(tc, sd, tn);

  // ---- pass 1: moments ------------------------------------------------------
  double acc[K + 1];
#pragma unroll
  for (int k = 0; k <= K; ++k) acc[k] = 0.0;
  {
    auto flush = [&](int n, uint64_t own) __attribute__((always_inline)) {
      int j, p;
      const bool act = item_of(n, j, p);
      PixelBasis pp;
      pp.tc = from_lane(pb.tc, p);
      pp.p = from_lane(pb.p, p);
      pp.p15 = from_lane(pb.p15, p);
      pp.amp = from_lane(pb.amp, p);
      const float lamp = from_lane(lam, p);
      double* resd = reinterpret_cast<double*>(res);
      if (act) {
        RayG g = ray_of(j, p, lamp);
        if constexpr (kTrig) {
          double m[K + 1];
          particle_trig_moments_d<NH>(g, tn, m);
#pragma unroll
          for (int k = 0; k <= K; ++k) resd[k * 64 + lane] = m[k];
        } else if constexpr (kDblMom) {
          double m[K + 1];
          particle_moments_d<K>(g, pp, tn, m);
#pragma unroll
          for (int k = 0; k <= K; ++k) resd[k * 64 + lane] = m[k];
        } else {
          float m[K + 1];
          particle_moments<K>(g, pp, tn, m);
#pragma unroll
          for (int k = 0; k <= K; ++k) res[k * 64 + lane] = m[k];
        }
      }
      __builtin_amdgcn_wave_barrier();
      while (own) {
        const int i = __builtin_ctzll(own);
        own &= own - 1;
#pragma unroll
        for (int k = 0; k <= K; ++k) acc[k] += kDblMom ? resd[k * 64 + i] : (double)res[k * 64 + i];
      }
      __builtin_amdgcn_wave_barrier();
    };
    for (int b = rg.x; b < rg.y; b += kBlock) {
      int nb = min(kBlock, rg.y - b);
      __syncthreads();
      load_batch_covered(st, a.rec, a.sorted_rec, a.masks, bw.quad, b, nb);
      __syncthreads();
      QueueCursor qc;
      queue_reset(qc);
      queue_from_masks<true>(q, qc, a.masks, b, nb, quad, own4, lane, ~0ull,
                       [&]() __attribute__((always_inline)) {
                         flush(64, qc.own_lo);
                         queue_pop64(q, qc, lane);
                       },
                       [](int) {});
      if (qc.cnt > 0) flush(qc.cnt, qc.own_lo);
    }
  }

  if (split) {
    double* xd = reinterpret_cast<double*>(&st);
    __syncthreads();
#pragma unroll
    for (int k = 0; k <= K; ++k) xd[(wave * (K + 1) + k) * 64 + lane] = acc[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k <= K; ++k) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < 4; ++w) t += xd[(w * (K + 1) + k) * 64 + lane];
      acc[k] = t;
    }
  }
  // the backward pass starts from these sums (one column per moment)
  if (inside && own4 <= 0) {
#pragma unroll
    for (int k = 0; k <= K; ++k) a.pix_mom[(size_t)k * a.n_pix + pix] = acc[k];
  }

  // ---- per-pixel setup ------------------------------------------------------
  const float m0 = (float)acc[0];
  // a pixel whose optical depth is below kMinDepth is empty: its radiance
  // (about m0 times a colour) is negligible, and its moment vector is too close
  // to the float32 underflow range to define a measure
  const bool live = acc[0] > kMinDepth;
  LInv<NH> L;
  TrigLInv<kTrig ? NH : 1> TL;
  bool fallback = false;
  if constexpr (kTrig) {
    if (live) fallback = trig_factor<NH>(acc, TL) != 0.0;
#pragma unroll
    for (int i = 0; i < (NH + 1) * (NH + 2) / 2; ++i) L.l[i] = 0.f;
  } else if (live && MODE != kModeEmit && MODE != kModeTabSur) {
    double bn[K + 1], bmix[K + 1];
    bn[0] = 1.0;
#pragma unroll
    for (int k = 1; k <= K; ++k) bn[k] = acc[k] / acc[0];
    fallback = hankel_factor<NH>(bn, L, bmix) != 0.0;
  } else {
#pragma unroll
    for (int i = 0; i < (NH + 1) * (NH + 2) / 2; ++i) L.l[i] = 0.f;
  }

  float feat[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float smu = 0.f, ssig = 1.f;
  if constexpr (MODE == kModeHarvest || MODE == kModeEmit || MODE == kModeTabSur) {
    static_assert(K == 6, "the surrogate takes six moments");
    if (live) surrogate_features(acc, feat, smu, ssig);
  }

  // ---- tabulated schedule: the pixel's record (and the bounds' table) -------
  if constexpr (MODE == kModeTabPlain || MODE == kModeTabSur) {
    if constexpr (MODE == kModeTabPlain) {
      if (live) {
        const double mb = acc[1] / acc[0];
        const double var = acc[2] / acc[0] - mb * mb;
        smu = (float)mb;
        ssig = (float)(var > 0.0 ? sqrt(var) : 1.0);
      }
    }
    if (inside && own4 <= 0) {
      float* pf = a.pixfeat + pix * kPixFeat;
#pragma unroll
      for (int k = 0; k < 6; ++k) pf[k] = feat[k];
      pf[6] = live ? m0 : 0.f;
      pf[7] = tc;
      pf[8] = sd;
      // covering count, as -(count + 1) where the bounds' measure was degenerate
      pf[9] = fallback ? -(float)(n_cov + 1) : (float)n_cov;
      pf[10] = smu;
      pf[11] = ssig;
      if constexpr (MODE == kModeTabPlain) {
        // the moment bounds at the nodes y_g = mean + sd z_g
        const float dz = 2.f * kTabZ / (float)(a.tab_nodes - 1);
        float* tp = a.tab + pix * a.tab_nodes;
        for (int g = 0; g < a.tab_nodes; ++g)
          tp[g] = live ? bound_F<NH>(L, smu + ssig * (-kTabZ + dz * (float)g), a.beta) : 0.f;
      }
    }
    return;
  }

  // ---- surrogate query list: this tile's range, pixel by pixel --------------
  long long qbase = -1;
  if constexpr (MODE == kModeEmit) {
    const int nq = (inside && live) ? n_cov * NQ : 0;
    int inc = nq;  // inclusive scan over the wave, then over the 4 waves
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      int t = __shfl_up(inc, d, 64);
      if (lane >= d) inc += t;
    }
    if (lane == 63) s_scan[wave] = inc;
    __syncthreads();
    int off = inc - nq, tot = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      off += w < wave ? s_scan[w] : 0;
      tot += s_scan[w];
    }
    if (tid == 0) s_base = tot > 0 ? (long long)atomicAdd(a.q_count, (unsigned long long)tot) : 0;
    __syncthreads();
    const long long base = s_base;
    // past the capacity the tile's pixels get no queries; the counter still
    // reports the full request so the caller can size the list and retry.
    // A reservation that straddles the capacity fills its part below it with
    // a harmless query (pixel 0), so every slot below min(count, capacity)
    // names a pixel of the image.
    if (base + tot <= a.q_cap) {
      if (inside && live) qbase = base + off;
    } else {
      for (long long i = base + tid; i < a.q_cap; i += kBlock) {
        a.q_z[i] = 0.f;
        a.q_pix[i] = 0;
      }
    }
    if (inside) {
      float* pf = a.pixfeat + pix * kPixFeat;
#pragma unroll
      for (int k = 0; k < 6; ++k) pf[k] = feat[k];
      pf[6] = m0;
      pf[7] = tc;
      pf[8] = sd;
      pf[9] = (float)n_cov;
      a.pix_qbase[pix] = qbase;
    }
  }

  // ---- pass 2: quadrature (or the surrogate's query list) -------------------
  float sr = 0.f, sg = 0.f, sb = 0.f, so = 0.f, spen = 0.f;
  const bool want_pen = a.penalty != nullptr;
  if constexpr (MODE == kModeEmit) {
    int i_pair = 0;
    for (int b = rg.x; b < rg.y; b += kBlock) {
      int nb = min(kBlock, rg.y - b);
      __syncthreads();
      load_batch(st, a.rec, a.sorted_rec, b, nb);
      __syncthreads();
      // the pairs of the coverage masks pass 0 stored (their count is n_cov)
      for_each_masked(a.masks, b, nb, quad, lane, [&](int j, uint64_t m) __attribute__((always_inline)) {
        if (inside && live && ((m >> lane) & 1ull)) {
          const float dx = u - st.f[0][j].x, dy = v - st.f[0][j].y;
          RayG g = ray_params(st, j, dx, dy, lam);
          QEdges<NQ> e;
          quad_edges<NQ>(g, pb, tn, a, e);
          if (qbase >= 0) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
              const long long qi = qbase + (long long)i_pair * NQ + k;
              a.q_z[qi] = std_query(e.y[k], smu, ssig);
              a.q_pix[qi] = (int)pix;
            }
          }
          ++i_pair;
        }
      });
    }
    return;
  } else {
    float4* cb = reinterpret_cast<float4*>(res);  // [64]
    float* cpen = res + 256;                       // [64] consistency penalty
    const uint64_t live_mask = __ballot(inside && live);
    // evaluate queue positions [0, n) (one per lane), then add the results of
    // this lane's own positions (bits of `own`) in order
    auto flush = [&](int n, uint64_t own, int b) __attribute__((always_inline)) {
      const bool act = lane < n;
      const int it = act ? (int)q.item[lane] : lane;
      const int j = act ? (it >> 6) : 0;
      const int p = it & 63;
      PixelBasis pp;
      pp.tc = from_lane(pb.tc, p);
      pp.p = from_lane(pb.p, p);
      pp.p15 = from_lane(pb.p15, p);
      pp.amp = from_lane(pb.amp, p);
      LInv<NH> Lp;
      TrigLInv<kTrig ? NH : 1> TLp;
      if constexpr (kTrig) {
#pragma unroll
        for (int i = 0; i < (NH + 1) * (NH + 2) / 2; ++i) {
          TLp.re[i] = from_lane(TL.re[i], p);
          TLp.im[i] = from_lane(TL.im[i], p);
        }
      } else {
#pragma unroll
        for (int i = 0; i < (NH + 1) * (NH + 2) / 2; ++i) Lp.l[i] = from_lane(L.l[i], p);
      }
      const float m0p = from_lane(m0, p), lamp = from_lane(lam, p);
      float featp[6], smup = 0.f, ssigp = 1.f;
      if constexpr (MODE == kModeHarvest) {
#pragma unroll
        for (int f = 0; f < 6; ++f) featp[f] = from_lane(feat[f], p);
        smup = from_lane(smu, p);
        ssigp = from_lane(ssig, p);
      }
      if (act) {
        const int ppx = x0 + (p & 7), ppy = y0 + (p >> 3);
        const float dx = (float)ppx + 0.5f - st.f[0][j].x;
        const float dy = (float)ppy + 0.5f - st.f[0][j].y;
        RayG g = ray_params(st, j, dx, dy, lamp);
        QEdges<NQ> e;
        float qv;
        if constexpr (kTrig) {
          qv = particle_quadrature_trig<NH, NQ>(g, TLp, m0p, tn, a, e);
        } else {
          qv = particle_quadrature<NH, NQ>(g, pp, Lp, m0p, tn, a, e);
        }
        if constexpr (MODE == kModeHarvest) {
          const uint32_t rid = (uint32_t)a.sorted_rec[b + j];
          const size_t pixp = ((size_t)ci * c.height + ppy) * c.width + ppx;
#pragma unroll
          for (int k = 0; k < NQ; ++k) {
            const uint32_t h = mix_hash(a.seed, (uint32_t)pixp, rid * NQ + k);
            if ((float)(h >> 8) * (1.f / 16777216.f) < a.harvest_rate) {
              const int slot = atomicAdd(a.harvest_count, 1);
              if (slot < a.harvest_cap) {
                float* o = a.harvest + (size_t)slot * kHarvestStride;
#pragma unroll
                for (int f = 0; f < 6; ++f) o[f] = featp[f];
                o[6] = std_query(e.y[k], smup, ssigp);
                o[7] = m0p;
                o[8] = expf(-e.tau[k]);
                o[9] = __uint_as_float(h);
                o[10] = __int_as_float((int)pixp);
                o[11] = __int_as_float((int)(rid * NQ + k));
              }
            }
          }
        }
        float4 f5 = st.f[5][j];
        cb[lane] = make_float4(qv * f5.y, qv * f5.z, qv * f5.w, qv);
        if (want_pen) cpen[lane] = pair_penalty<NQ>(g, tn, e, a);
      }
      __builtin_amdgcn_wave_barrier();
      while (own) {
        const int i = __builtin_ctzll(own);
        own &= own - 1;
        const float4 c4 = cb[i];
        sr += c4.x;
        sg += c4.y;
        sb += c4.z;
        so += c4.w;
        if (want_pen) spen += cpen[i];
      }
      __builtin_amdgcn_wave_barrier();
    };
    for (int b = rg.x; b < rg.y; b += kBlock) {
      int nb = min(kBlock, rg.y - b);
      __syncthreads();
      load_batch_covered(st, a.rec, a.sorted_rec, a.masks, bw.quad, b, nb);
      __syncthreads();
      QueueCursor qc;
      queue_reset(qc);
      queue_from_masks<true>(q, qc, a.masks, b, nb, quad, own4, lane, live_mask,
                       [&]() __attribute__((always_inline)) {
                         flush(64, qc.own_lo, b);
                         queue_pop64(q, qc, lane);
                       },
                       [](int) {});
      if (qc.cnt > 0) flush(qc.cnt, qc.own_lo, b);
    }
  }

  if (split) {
    __syncthreads();
    xch[(wave * 5 + 0) * 64 + lane] = sr;
    xch[(wave * 5 + 1) * 64 + lane] = sg;
    xch[(wave * 5 + 2) * 64 + lane] = sb;
    xch[(wave * 5 + 3) * 64 + lane] = so;
    xch[(wave * 5 + 4) * 64 + lane] = spen;
    __syncthreads();
    sr = sg = sb = so = spen = 0.f;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      sr += xch[(w * 5 + 0) * 64 + lane];
      sg += xch[(w * 5 + 1) * 64 + lane];
      sb += xch[(w * 5 + 2) * 64 + lane];
      so += xch[(w * 5 + 3) * 64 + lane];
      spen += xch[(w * 5 + 4) * 64 + lane];
    }
    if (wave != 0) return;
  }

  // ---- epilogue: Eq. 15 ------------------------------------------------------
  if (!inside) return;
  float alpha = -expm1f(-m0);
  float tr = expf(-m0);
  float inv_o = 1.f / fmaxf(a.eps, so);
  float* out = a.image + pix * 3;
  out[0] = alpha * sr * inv_o + tr * c.bg[0];
  out[1] = alpha * sg * inv_o + tr * c.bg[1];
  out[2] = alpha * sb * inv_o + tr * c.bg[2];
  float4* sv = reinterpret_cast<float4*>(a.saved + pix * MB_SAVED_FLOATS_PER_PIXEL);
  sv[0] = make_float4(sr, sg, sb, so);
  if (want_pen) a.penalty[pix] = spen;
  // covering count; stored as -(count + 1) when the pixel's measure was
  // degenerate (mixed with a normal, or the identity factor; see hankel_factor)
  sv[1] = make_float4(tc, sd, m0, fallback ? -(float)(n_cov + 1) : (float)n_cov);
}

// Second half of the surrogate forward: Eq. 7 with the optical depth m_0 F
// from the surrogate's outputs for the queries the emit pass listed, in the
// same pair order (query index = pixel base + pair * NQ + edge).
template <int NQ>
__global__ __launch_bounds__(256) void k_render_consume(RenderArgs a, CamSet cams) {
  __shared__ Stage st;
  const int tiles_per_cam = a.tiles_x * a.tiles_y;
  const int n_keys = tiles_per_cam * a.n_cams;
  const int key = block_work(a).key;  // the surrogate path splits no tile
  if (key >= n_keys) return;
  const int ci = key / tiles_per_cam;
  const int tile = key - ci * tiles_per_cam;
  const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
  const CamConst& c = cams.c[ci];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int px = tx * kTile + (wave & 1) * 8 + (lane & 7);
  const int py = ty * kTile + (wave >> 1) * 8 + (lane >> 3);
  const bool inside = px < c.width && py < c.height;
  const float u = (float)px + 0.5f, v = (float)py + 0.5f;
  const float rx = (u - c.cx) / c.fx, ry = (v - c.cy) / c.fy;
  const float lam = sqrtf(1.f + rx * rx + ry * ry);
  const float tn = c.tn;
  const int2 rg = a.ranges[key];
  const size_t pix = ((size_t)ci * c.height + (inside ? py : 0)) * c.width + (inside ? px : 0);
  const float* pf = a.pixfeat + pix * kPixFeat;
  const float m0 = inside ? pf[6] : 0.f;
  const long long qbase = inside ? a.pix_qbase[pix] : -1;
  const bool active = qbase >= 0;
  const PixelBasis pb = make_basis(inside ? pf[7] : tn, inside ? pf[8] : 1.f, tn);
  float sr = 0.f, sg = 0.f, sb = 0.f, so = 0.f;
  int i_pair = 0;
  for (int b = rg.x; b < rg.y; b += kBlock) {
    int nb = min(kBlock, rg.y - b);
    __syncthreads();
    load_batch(st, a.rec, a.sorted_rec, b, nb);
    __syncthreads();
    // the pairs of the forward pass's coverage masks, in the emit pass's order
    for_each_masked(a.masks, b, nb, wave, lane, [&](int j, uint64_t m) __attribute__((always_inline)) {
      if (active && ((m >> lane) & 1ull)) {
        const float dx = u - st.f[0][j].x, dy = v - st.f[0][j].y;
        RayG g = ray_params(st, j, dx, dy, lam);
        QEdges<NQ> e;
        quad_edges<NQ>(g, pb, tn, a, e);
        const float* fq = a.q_f + qbase + (long long)i_pair * NQ;
        // the bounds the surrogate stands for grow with depth: its optical
        // depth along the edges is made non-decreasing (running maximum; a
        // later edge takes over only when strictly larger)
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
          const float tk = m0 * fq[k];
          e.tau[k] = (k == 0 || tk > e.tau[k > 0 ? k - 1 : 0]) ? tk : e.tau[k > 0 ? k - 1 : 0];
        }
        float q = quad_sum<NQ>(g, tn, e);
        float4 f5 = st.f[5][j];
        sr += q * f5.y;
        sg += q * f5.z;
        sb += q * f5.w;
        so += q;
        ++i_pair;
      }
    });
  }
  if (!inside) return;
  float alpha = -expm1f(-m0);
  float tr = expf(-m0);
  float inv_o = 1.f / fmaxf(a.eps, so);
  float* out = a.image + pix * 3;
  out[0] = alpha * sr * inv_o + tr * c.bg[0];
  out[1] = alpha * sg * inv_o + tr * c.bg[1];
  out[2] = alpha * sb * inv_o + tr * c.bg[2];
  float4* sv = reinterpret_cast<float4*>(a.saved + pix * MB_SAVED_FLOATS_PER_PIXEL);
  sv[0] = make_float4(sr, sg, sb, so);
  sv[1] = make_float4(pf[7], pf[8], m0, pf[9]);
}

// Second half of the tabulated schedule: Eq. 7 and Eq. 15 with the optical
// depth at every edge interpolated linearly in the pixel's table at the
// edge's standardised query (clamped to the table's ends), made
// non-decreasing along the edges (a running maximum; the surrogate's table
// need not grow, the bounds' table does).
template <int NQ>
__global__ __launch_bounds__(256) void k_render_consume_tab(RenderArgs a, CamSet cams) {
  __shared__ Stage st;
  __shared__ WaveQueue wq[4];
  __shared__ __align__(16) float4 wres[4][64];
  const int tiles_per_cam = a.tiles_x * a.tiles_y;
  const int n_keys = tiles_per_cam * a.n_cams;
  const int key = block_work(a).key;  // the tabulated schedule splits no tile
  if (key >= n_keys) return;
  const int ci = key / tiles_per_cam;
  const int tile = key - ci * tiles_per_cam;
  const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
  const CamConst& c = cams.c[ci];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int x0 = tx * kTile + (wave & 1) * 8, y0 = ty * kTile + (wave >> 1) * 8;
  const int px = x0 + (lane & 7), py = y0 + (lane >> 3);
  const bool inside = px < c.width && py < c.height;
  const float u = (float)px + 0.5f, v = (float)py + 0.5f;
  const float rx = (u - c.cx) / c.fx, ry = (v - c.cy) / c.fy;
  const float lam = sqrtf(1.f + rx * rx + ry * ry);
  const float tn = c.tn;
  const int2 rg = a.ranges[key];
  const size_t pix = ((size_t)ci * c.height + (inside ? py : 0)) * c.width + (inside ? px : 0);
  const float* pf = a.pixfeat + pix * kPixFeat;
  const float m0 = inside ? pf[6] : 0.f;
  const bool active = inside && m0 > 0.f;
  const PixelBasis pb = make_basis(inside ? pf[7] : tn, inside ? pf[8] : 1.f, tn);
  const float smu = inside ? pf[10] : 0.f, isig = inside ? 1.f / pf[11] : 1.f;
  const float ucoef = (float)(a.tab_nodes - 1) / (2.f * kTabZ);
  const uint64_t active_mask = __ballot(active);
  WaveQueue& q = wq[wave];
  float4* res = wres[wave];
  float sr = 0.f, sg = 0.f, sb = 0.f, so = 0.f;
  // as the quadrature pass of k_render_fwd: covering pairs evaluated 64 at a
  // time, one per lane, the results added by the pixel's own lane in list order
  auto flush = [&](int n, uint64_t own) __attribute__((always_inline)) {
    const bool act = lane < n;
    const int it = act ? (int)q.item[lane] : lane;
    const int j = act ? (it >> 6) : 0;
    const int p = it & 63;
    PixelBasis pp;
    pp.tc = from_lane(pb.tc, p);
    pp.p = from_lane(pb.p, p);
    pp.p15 = from_lane(pb.p15, p);
    pp.amp = from_lane(pb.amp, p);
    const float m0p = from_lane(m0, p), lamp = from_lane(lam, p);
    const float smup = from_lane(smu, p), isigp = from_lane(isig, p);
    if (act) {
      const int ppx = x0 + (p & 7), ppy = y0 + (p >> 3);
      const float dx = (float)ppx + 0.5f - st.f[0][j].x;
      const float dy = (float)ppy + 0.5f - st.f[0][j].y;
      RayG g = ray_params(st, j, dx, dy, lamp);
      QEdges<NQ> e;
      quad_edges<NQ>(g, pp, tn, a, e);
      const float* tp = a.tab + (((size_t)ci * c.height + ppy) * c.width + ppx) * a.tab_nodes;
#pragma unroll
      for (int k = 0; k < NQ; ++k) {
        const float z = fminf(fmaxf((e.y[k] - smup) * isigp, -kTabZ), kTabZ);
        const float uu = (z + kTabZ) * ucoef;
        const int i0 = min((int)uu, a.tab_nodes - 2);
        const float fr = uu - (float)i0;
        const float f = fmaf(fr, tp[i0 + 1] - tp[i0], tp[i0]);
        const float tk = m0p * f;
        e.tau[k] = (k == 0 || tk > e.tau[k > 0 ? k - 1 : 0]) ? tk : e.tau[k > 0 ? k - 1 : 0];
      }
      const float qv = quad_sum<NQ>(g, tn, e);
      const float4 f5 = st.f[5][j];
      res[lane] = make_float4(qv * f5.y, qv * f5.z, qv * f5.w, qv);
    }
    __builtin_amdgcn_wave_barrier();
    while (own) {
      const int i = __builtin_ctzll(own);
      own &= own - 1;
      const float4 c4 = res[i];
      sr += c4.x;
      sg += c4.y;
      sb += c4.z;
      so += c4.w;
    }
    __builtin_amdgcn_wave_barrier();
  };
  for (int b = rg.x; b < rg.y; b += kBlock) {
    int nb = min(kBlock, rg.y - b);
    __syncthreads();
    load_batch_covered(st, a.rec, a.sorted_rec, a.masks, -1, b, nb);
    __syncthreads();
    QueueCursor qc;
    queue_reset(qc);
    queue_from_masks<true>(q, qc, a.masks, b, nb, wave, -1, lane, active_mask,
                           [&]() __attribute__((always_inline)) {
                             flush(64, qc.own_lo);
                             queue_pop64(q, qc, lane);
                           },
                           [](int) {});
    if (qc.cnt > 0) flush(qc.cnt, qc.own_lo);
  }
  if (!inside) return;
  float alpha = -expm1f(-m0);
  float tr = expf(-m0);
  float inv_o = 1.f / fmaxf(a.eps, so);
  float* out = a.image + pix * 3;
  out[0] = alpha * sr * inv_o + tr * c.bg[0];
  out[1] = alpha * sg * inv_o + tr * c.bg[1];
  out[2] = alpha * sb * inv_o + tr * c.bg[2];
  float4* sv = reinterpret_cast<float4*>(a.saved + pix * MB_SAVED_FLOATS_PER_PIXEL);
  sv[0] = make_float4(sr, sg, sb, so);
  sv[1] = make_float4(pf[7], pf[8], m0, pf[9]);
}

hipError_t launch_render_consume_tab(const RenderArgs& a, const CamSet& cams, int n_intervals, hipStream_t s) {
  int n_keys = a.tiles_x * a.tiles_y * a.n_cams;
  dim3 grid(render_blocks(n_keys)), block(kBlock);
  if (n_intervals == 3)
    hipLaunchKernelGGL(k_render_consume_tab<4>, grid, block, 0, s, a, cams);
  else if (n_intervals == 5)
    hipLaunchKernelGGL(k_render_consume_tab<6>, grid, block, 0, s, a, cams);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_render_forward(const RenderArgs& a, const CamSet& cams, int n_moments, int n_intervals,
                                 hipStream_t s, int mode) {
  int n_keys = a.tiles_x * a.tiles_y * a.n_cams;
  dim3 grid(render_blocks(n_keys)), block(kBlock);
#define MB_LAUNCH(KK, NN, MM)                                                       \
  if (n_moments == KK && n_intervals == NN && mode == MM) {                         \
    hipLaunchKernelGGL((k_render_fwd<KK, NN + 1, MM>), grid, block, 0, s, a, cams); \
    return hipGetLastError();                                                       \
  }
  MB_LAUNCH(4, 3, kModePlain)
  MB_LAUNCH(6, 3, kModePlain)
  MB_LAUNCH(4, 5, kModePlain)
  MB_LAUNCH(6, 5, kModePlain)
  MB_LAUNCH(8, 3, kModePlain)
  MB_LAUNCH(8, 5, kModePlain)
  MB_LAUNCH(6, 3, kModeHarvest)
  MB_LAUNCH(6, 5, kModeHarvest)
  MB_LAUNCH(6, 3, kModeEmit)
  MB_LAUNCH(6, 5, kModeEmit)
  MB_LAUNCH(4, 3, kModeTrig)
  MB_LAUNCH(4, 5, kModeTrig)
  MB_LAUNCH(6, 3, kModeTrig)
  MB_LAUNCH(6, 5, kModeTrig)
  MB_LAUNCH(4, 3, kModeTabPlain)
  MB_LAUNCH(6, 3, kModeTabPlain)
  MB_LAUNCH(4, 5, kModeTabPlain)
  MB_LAUNCH(6, 5, kModeTabPlain)
  MB_LAUNCH(6, 3, kModeTabSur)
  MB_LAUNCH(6, 5, kModeTabSur)
#undef MB_LAUNCH
  return hipErrorInvalidValue;
}

hipError_t launch_render_consume(const RenderArgs& a, const CamSet& cams, int n_intervals, hipStream_t s) {
  int n_keys = a.tiles_x * a.tiles_y * a.n_cams;
  dim3 grid(render_blocks(n_keys)), block(kBlock);
  if (n_intervals == 3)
    hipLaunchKernelGGL(k_render_consume<4>, grid, block, 0, s, a, cams);
  else if (n_intervals == 5)
    hipLaunchKernelGGL(k_render_consume<6>, grid, block, 0, s, a, cams);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace mb
