// Backward render: the two-stage adjoint of Sec. 3.3 (Eq. 22, App. D), one
// workgroup per 16x16 tile as in the forward pass.
//   pass 1   the pixel's moment sums, as the forward pass stored them (per
//            pixel; nothing per (pixel, Gaussian) pair is stored);
//   setup    Hankel factor; the derivative of the Eq. 15 rescaling is folded
//            in: a = g (1 - e^-m0) / max(eps, O), b = dL/dO, e0 = dL/dm0;
//   pass 2   Adjoint-Moment stage: dm = e0 e_0 + sum_i (a . c_i + b) dq_i/dm,
//            through the quadrature (Eq. 7) and the adjoint of the moment
//            bounds at every interval edge; the same evaluation also gives
//            the part of the Gradient stage that does not depend on dm,
//            (a . c_i + b) dq_i/dtheta_i for theta = (mu, Sigma, omega) and the
//            colour term, chained to the record coefficients;
//   pass 3   the rest of the Gradient stage, dm . dm_i/dtheta_i.
// Per-pair gradients are summed over the wave's pixels into one slot per
// (list entry, wave) (pass 2 writes it, pass 3 adds to it); a per-Gaussian
// kernel then sums the slots: one reduction, no atomics, deterministic. A
// byte per slot records whether it was written (the stored coverage mask of
// that entry and quadrant is non-empty); the reduction skips the others.
// The passes walk the coverage masks the forward pass stored.
#include "render_common.h"
#include "trig.h"

namespace mb {

// Quadrature of one Gaussian with the state its adjoint needs.
template <int NH, int NQ>
struct QuadState {
  float t[NQ], y[NQ], w0[NQ], F[NQ], tau[NQ], T[NQ], sr[NQ], off[NQ];
  float x[NQ][NH];
  bool below[NQ][NH];
  bool cl[NQ];
  float dt[NQ], ph[NQ], dph[NQ], A[NQ];
  float q;
};

// phi'(x) = (e^-x - phi(x)) / x from d = e^-x and phi: the derivative of
// phi's series (terms up to x^4) for |x| < 1/16, the direct form beyond
__device__ __forceinline__ float dphi_fn(float x, float d, float ph) {
  // coefficients (-1)^k k / (k+1)!, k = 1..5
  float s = 5.f / 720.f;
  s = fmaf(s, -x, 4.f / 120.f);
  s = fmaf(s, -x, 3.f / 24.f);
  s = fmaf(s, -x, 2.f / 6.f);
  s = fmaf(s, -x, 0.5f);
  return fabsf(x) < kPhiSeries ? -s : (d - ph) * fast_rcp(x);
}

// Edges of one Gaussian's quadrature (App. B) and sigma_i there.
template <int NH, int NQ>
__device__ __forceinline__ void quad_geom(const RayG& g, const PixelBasis& pb, float tn, const RenderArgs& a,
                                          QuadState<NH, NQ>& s) {
  float dtc = g.mu - pb.tc;
  const float rn = (tn - g.mu) * fast_rcp(g.sig);  // edges moved onto the near bound
  const float en = exp_neg_half(rn * rn);
#pragma unroll
  for (int j = 0; j < NQ; ++j) {
    s.off[j] = a.kappa * g.sig * a.xq[j];
    float t = g.mu + s.off[j];
    s.cl[j] = t < tn;
    float dtj = s.cl[j] ? (tn - pb.tc) : (dtc + s.off[j]);
    s.t[j] = s.cl[j] ? tn : t;
    s.y[j] = warp_y(pb, s.t[j], dtj);
    s.sr[j] = s.cl[j] ? en : a.eq[j];
  }
}

// Given the optical depth s.tau at the edges: the Eq. 7 terms, q, and
// A[j] = dq / dtau_j.
template <int NH, int NQ>
__device__ __forceinline__ void quad_terms(const RayG& g, float tn, QuadState<NH, NQ>& s) {
  s.T[0] = __expf(-s.tau[0]);
  s.q = 0.f;
#pragma unroll
  for (int j = 0; j < NQ; ++j) s.A[j] = 0.f;
#pragma unroll
  for (int j = 0; j + 1 < NQ; ++j) {
    s.dt[j] = s.cl[j + 1] ? 0.f : (s.cl[j] ? (g.mu + s.off[j + 1] - tn) : (s.off[j + 1] - s.off[j]));
    float dtau = s.tau[j + 1] - s.tau[j];
    const float d = __expf(-dtau);
    s.T[j + 1] = s.T[j] * d;
    s.ph[j] = phi_fn(dtau, d);
    s.dph[j] = dphi_fn(dtau, d, s.ph[j]);
    float tds = s.T[j] * s.dt[j] * g.omega * s.sr[j];
    s.q += tds * s.ph[j];
    // dq/dtau_j and dq/dtau_{j+1} of this interval's term
    s.A[j] -= tds * (s.ph[j] + s.dph[j]);
    s.A[j + 1] += tds * s.dph[j];
  }
}

template <int NH, int NQ>
__device__ __forceinline__ void quad_state(const RayG& g, const PixelBasis& pb, const LInv<NH>& L, float m0,
                                           float tn, const RenderArgs& a, QuadState<NH, NQ>& s) {
  quad_geom<NH, NQ>(g, pb, tn, a, s);
#pragma unroll
  for (int j = 0; j < NQ; ++j) {
    s.F[j] = canon_at<NH>(L, s.y[j], a.beta, s.x[j], s.below[j], s.w0[j]);
    s.tau[j] = m0 * s.F[j];
  }
  quad_terms<NH, NQ>(g, tn, s);
}

// The same for the trigonometric moments (the forward pass's
// particle_quadrature_trig): the edge at depth t queries the angle
// psi = (2 pi - theta) g_hat(t) (kept in s.y), the optical depth is a running
// maximum along the edges, and src[e] names the edge whose query supplied
// edge e's value (the last edge at or before e that raised it).
template <int NH, int NQ>
__device__ __forceinline__ void trig_quad_state(const RayG& g, const TrigLInv<NH>& L, float m0, float tn,
                                                const RenderArgs& a, QuadState<NH, NQ>& s, TrigCanon<NH>* tc,
                                                int* src) {
  cfl start = {__builtin_nanf(""), 0.f};  // the first edge starts from its query point
#pragma unroll
  for (int j = 0; j < NQ; ++j) {
    s.off[j] = a.kappa * g.sig * a.xq[j];
    const float t = g.mu + s.off[j];
    s.cl[j] = t < tn;
    s.t[j] = s.cl[j] ? tn : t;
    s.y[j] = kTrigSpan * warp_abs(s.t[j], tn);
    const float r = (s.t[j] - g.mu) * fast_rcp(g.sig);
    s.sr[j] = s.cl[j] ? exp_neg_half(r * r) : a.eq[j];
    s.F[j] = trig_canon<NH>(L, s.y[j], a.beta, tc[j], &start);
    const float tj = m0 * s.F[j];
    const bool up = j == 0 || tj > s.tau[j > 0 ? j - 1 : 0];
    s.tau[j] = up ? tj : s.tau[j > 0 ? j - 1 : 0];
    src[j] = up ? j : src[j > 0 ? j - 1 : 0];
  }
  quad_terms<NH, NQ>(g, tn, s);
}

// Double-precision dual number (one tangent) for the Jacobian of the
// surrogate's inputs with respect to the pixel's moments.
struct DualD {
  double v, d;
  __device__ DualD(double a = 0.0, double b = 0.0) : v(a), d(b) {}
};
__device__ __forceinline__ DualD operator+(DualD a, DualD b) { return DualD(a.v + b.v, a.d + b.d); }
__device__ __forceinline__ DualD operator-(DualD a, DualD b) { return DualD(a.v - b.v, a.d - b.d); }
__device__ __forceinline__ DualD operator*(DualD a, DualD b) { return DualD(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ __forceinline__ DualD operator/(DualD a, DualD b) {
  double r = a.v / b.v;
  return DualD(r, (a.d - r * b.d) / b.v);
}

// Surrogate inputs as functions of the pixel's moments m_0..m_6, as in the
// forward pass: asinh of the standardised moments 1..6 of b = m / m_0, and
// the standardisation (mean mu, standard deviation sig) of the moment variable.
__device__ __forceinline__ void feat_from_moments(const DualD* m, DualD* feat, DualD& mu, DualD& sig) {
  DualD b[7];
  b[0] = DualD(1.0);
#pragma unroll
  for (int k = 1; k <= 6; ++k) b[k] = m[k] / m[0];
  mu = b[1];
  DualD var = b[2] - mu * mu;
  if (var.v > 0.0) {
    const double sq = sqrt(var.v);
    sig = DualD(sq, 0.5 * var.d / sq);
  } else {
    sig = DualD(1.0);
  }
  const DualD is = DualD(1.0) / sig;
  DualD sk(1.0);
#pragma unroll
  for (int k = 1; k <= 6; ++k) {
    DualD c(0.0), pw(1.0);
    double binom = 1.0;
#pragma unroll
    for (int j = k; j >= 0; --j) {
      c = c + DualD(binom) * b[j] * pw;
      binom = binom * (double)j / (double)(k - j + 1);
      pw = pw * (DualD(0.0) - mu);
    }
    sk = sk * is;
    const DualD u = c * sk;
    feat[k - 1] = DualD(asinh(u.v), u.d / sqrt(1.0 + u.v * u.v));
  }
}

// sum_k dm[k] * d m_k / d(mu, Sigma, omega) for the moments of Eqs. 10-12,
// by reverse-mode differentiation of their recurrence: the moments forward
// (kept in registers), then one adjoint sweep back through the recurrence to
// the shared terms G, G', bn, E, erfc, and from those to (mu, Sigma, omega).
template <int K>
__device__ __forceinline__ void moment_grads(const RayG& g, const PixelBasis& pb, float tn, const float* dmv,
                                             float* out) {
  const float c = kSqrtHalfPi;
  const float mus = fmaxf(g.mu, tn);
  const float ys = warp_y(pb, mus, mus - pb.tc);
  const float Gp = warp_dy(pb, mus);
  const float G = ys + Gp * (g.mu - mus);
  const float q = 1.f + 0.8f * g.mu;
  const float d2 = g.mu > tn ? -3.f * pb.amp * fast_rcp(q * q * q * fast_sqrt(q)) : 0.f;  // y''(mu)
  const float is = fast_rcp(g.sig);
  const float bn = (tn - g.mu) * kInvSqrt2 * is;
  const float E = __expf(-bn * bn);
  const float ec = erfc_fast(bn);
  const float s2 = g.sig * g.sig;
  const float tm = tn - g.mu;
  // primal: m_0, m_1 and m_k = G m_{k-1} + (k-1) v2 m_{k-2} + bnd un^(k-1)
  float m[K + 1], up[K];
  m[0] = g.omega * g.sig * c * ec;
  const float bnd = Gp * g.omega * s2 * E;
  m[1] = G * m[0] + bnd;
  const float un = G + Gp * tm;
  const float v2 = Gp * Gp * s2;
  up[0] = 1.f;
#pragma unroll
  for (int k = 1; k < K; ++k) up[k] = up[k - 1] * un;
#pragma unroll
  for (int k = 2; k <= K; ++k) m[k] = G * m[k - 1] + (float)(k - 1) * v2 * m[k - 2] + bnd * up[k - 1];
  // adjoint sweep
  float a[K + 1];
#pragma unroll
  for (int k = 0; k <= K; ++k) a[k] = dmv[k];
  float gG = 0.f, gv2 = 0.f, gbnd = 0.f, gun = 0.f;
#pragma unroll
  for (int k = K; k >= 2; --k) {
    const float km = (float)(k - 1);
    gG += a[k] * m[k - 1];
    a[k - 1] += a[k] * G;
    gv2 += a[k] * km * m[k - 2];
    a[k - 2] += a[k] * km * v2;
    gbnd += a[k] * up[k - 1];
    gun += a[k] * km * up[k - 2];
  }
  gun *= bnd;
  gG += a[1] * m[0] + gun;
  a[0] += a[1] * G;
  gbnd += a[1];
  float gGp = gun * tm + gv2 * 2.f * Gp * s2 + gbnd * g.omega * s2 * E;
  float gmu = -gun * Gp;
  const float gs2 = gv2 * Gp * Gp + gbnd * Gp * g.omega * E;
  const float gE = gbnd * Gp * g.omega * s2;
  float gom = gbnd * Gp * s2 * E + a[0] * g.sig * c * ec;
  float gsig = a[0] * g.omega * c * ec + gs2 * 2.f * g.sig;
  const float gec = a[0] * g.omega * g.sig * c;
  const float gbn = -2.f * E * (gE * bn + gec * 0.5641895835477563f);  // d erfc/db = -2 E / sqrt(pi)
  gmu += -gbn * kInvSqrt2 * is + gG * Gp + gGp * d2;
  gsig += -gbn * bn * is;
  out[0] = gmu;
  out[1] = gsig;
  out[2] = gom;
}

struct BwdArgs {
  RenderArgs r;
  const float* saved;       // [C,H,W,8]
  const float* grad_image;  // [C,H,W,3]
  const float* grad_penalty;  // [C,H,W] dL/d(consistency penalty), or null
  const int* sorted_k;      // [E] entry index of each sorted list position
  float* partials;          // [E,4,kGradStride]
  uint8_t* used;            // [E,4]: which of an entry's slots this pass writes
};

// (mu, Sigma, omega) gradients of one pair -> gradients of its record
// coefficients (the inverse of ray_params); linear in (gmu, gsig, gom)
__device__ __forceinline__ void chain_record(float gmu, float gsig, float gom, const RayG& g, float lamp, float dx,
                                             float dy, const float4& f2, const float4& f3, const float4& f4,
                                             float* gr) {
  // D, X and the exponential as ray_params evaluated them at this offset
  const float id = g.id, ek = g.ek;
  float gE = gmu * lamp * id;
  float gD = -gmu * g.mu * id - 0.5f * gsig * g.sig * id + 0.5f * gom * g.omega * g.xid * id;
  float gX = -0.5f * gom * g.omega * id;
  gr[G_D0] = gD;
  gr[G_D1X] = 2.f * gD * dx;
  gr[G_D1Y] = 2.f * gD * dy;
  gr[G_D2XX] = gD * dx * dx;
  gr[G_D2XY] = 2.f * gD * dx * dy;
  gr[G_D2YY] = gD * dy * dy;
  gr[G_E0] = gE;
  gr[G_EX] = gE * dx;
  gr[G_EY] = gE * dy;
  gr[G_XXX] = gX * dx * dx;
  gr[G_XXY] = 2.f * gX * dx * dy;
  gr[G_XYY] = gX * dy * dy;
  float gdx = 2.f * gD * (f2.y + f2.w * dx + f3.x * dy) + gE * f3.w + 2.f * gX * (f4.y * dx + f4.z * dy);
  float gdy = 2.f * gD * (f2.z + f3.x * dx + f3.y * dy) + gE * f4.x + 2.f * gX * (f4.z * dx + f4.w * dy);
  gr[G_P0X] = -gdx;
  gr[G_P0Y] = -gdy;
  gr[G_W] = gom * ek;
}

// Segmented inclusive scan over the wave's lanes with DPP moves: four
// shifts inside each 16-lane row (row_shr 1, 2, 4, 8), then the classic
// row_bcast 15 (rows 1 and 3) and row_bcast 31 (rows 2 and 3) steps across
// rows. Each step adds the moved value times a 0/1 mask that keeps the sum
// inside the lane's segment [seg_start, lane]; the masks depend only on the
// segment layout, so one set serves every gradient field. The segment's last
// lane ends with the segment sum.
struct ScanMasks {
  float m[6];
};
__device__ __forceinline__ ScanMasks scan_masks(int lane, int seg_start) {
  ScanMasks s;
  const int row0 = lane & ~15;
  const int lo = max(seg_start, row0);
  s.m[0] = lane - 1 >= lo ? 1.f : 0.f;
  s.m[1] = lane - 2 >= lo ? 1.f : 0.f;
  s.m[2] = lane - 4 >= lo ? 1.f : 0.f;
  s.m[3] = lane - 8 >= lo ? 1.f : 0.f;
  s.m[4] = ((lane >> 4) & 1) && seg_start < row0 ? 1.f : 0.f;  // takes lane 15 or 47
  s.m[5] = (lane >> 5) && seg_start <= 31 ? 1.f : 0.f;         // takes lane 31
  return s;
}
// The scan of the gradient fields in one block of v_fmac_f32 with a DPP
// source (v += (v moved) * mask; the compiler would emit a separate move for
// each), step by step over the fields: all 18, or the 15 record fields when
// the colour fields are zero in every lane (the moment part of the Gradient
// stage). A DPP read of a VGPR written by a VALU instruction needs two wait
// states: within the block every read comes 15 or more instructions after
// the write it depends on, and the s_nop covers the values written just
// before the block.
static_assert(G_COUNT == 18 && G_CR == 15, "the scan blocks are written for 15 record and 3 colour fields");
#define MB_SCAN15(M, CTRL) \
  "v_fmac_f32_dpp %0, %0, " M " " CTRL "\n\t" \
  "v_fmac_f32_dpp %1, %1, " M " " CTRL "\n\t" \
  "v_fmac_f32_dpp %2, %2, " M " " CTRL "\n\t" \
  "v_fmac_f32_dpp %3, %3, " M " " CTRL "\n\t" \
  "v_fmac_f32_dpp %4, %4, " M " " CTRL "\n\t" \
  "v_fmac_f32_dpp %5, %5, " M " " CTRL "\n\t" \
  "v_fmac_f32_dpp %6, %6, " M " " CTRL "\n\t" \
  "v_fmac_f32_dpp %7, %7, " M " " CTRL "\n\t" \
  "v_fmac_f32_dpp %8, %8, " M " " CTRL "\n\t" \
  "v_fmac_f32_dpp %9, %9, " M " " CTRL "\n\t" \
  "v_fmac_f32_dpp %10, %10, " M " " CTRL "\n\t" \
  "v_fmac_f32_dpp %11, %11, " M " " CTRL "\n\t" \
  "v_fmac_f32_dpp %12, %12, " M " " CTRL "\n\t" \
  "v_fmac_f32_dpp %13, %13, " M " " CTRL "\n\t" \
  "v_fmac_f32_dpp %14, %14, " M " " CTRL "\n\t"
#define MB_SCAN18(M, CTRL) \
  MB_SCAN15(M, CTRL) \
  "v_fmac_f32_dpp %15, %15, " M " " CTRL "\n\t" \
  "v_fmac_f32_dpp %16, %16, " M " " CTRL "\n\t" \
  "v_fmac_f32_dpp %17, %17, " M " " CTRL "\n\t"

#define MB_ROW(C) "row_shr:" C " row_mask:0xf bank_mask:0xf bound_ctrl:1"
#define MB_BCAST15 "row_bcast:15 row_mask:0xa bank_mask:0xf bound_ctrl:1"
#define MB_BCAST31 "row_bcast:31 row_mask:0xc bank_mask:0xf bound_ctrl:1"
__device__ __forceinline__ void segment_scan18(float* g, const ScanMasks& s) {
  asm("s_nop 1\n\t"
      MB_SCAN18("%18", MB_ROW("1"))
      MB_SCAN18("%19", MB_ROW("2"))
      MB_SCAN18("%20", MB_ROW("4"))
      MB_SCAN18("%21", MB_ROW("8"))
      MB_SCAN18("%22", MB_BCAST15)
      MB_SCAN18("%23", MB_BCAST31)
      : "+v"(g[0]), "+v"(g[1]), "+v"(g[2]), "+v"(g[3]), "+v"(g[4]), "+v"(g[5]), "+v"(g[6]), "+v"(g[7]),
        "+v"(g[8]), "+v"(g[9]), "+v"(g[10]), "+v"(g[11]), "+v"(g[12]), "+v"(g[13]), "+v"(g[14]),
        "+v"(g[15]), "+v"(g[16]), "+v"(g[17])
      : "v"(s.m[0]), "v"(s.m[1]), "v"(s.m[2]), "v"(s.m[3]), "v"(s.m[4]), "v"(s.m[5]));
}
__device__ __forceinline__ void segment_scan15(float* g, const ScanMasks& s) {
  asm("s_nop 1\n\t"
      MB_SCAN15("%15", MB_ROW("1"))
      MB_SCAN15("%16", MB_ROW("2"))
      MB_SCAN15("%17", MB_ROW("4"))
      MB_SCAN15("%18", MB_ROW("8"))
      MB_SCAN15("%19", MB_BCAST15)
      MB_SCAN15("%20", MB_BCAST31)
      : "+v"(g[0]), "+v"(g[1]), "+v"(g[2]), "+v"(g[3]), "+v"(g[4]), "+v"(g[5]), "+v"(g[6]), "+v"(g[7]),
        "+v"(g[8]), "+v"(g[9]), "+v"(g[10]), "+v"(g[11]), "+v"(g[12]), "+v"(g[13]), "+v"(g[14])
      : "v"(s.m[0]), "v"(s.m[1]), "v"(s.m[2]), "v"(s.m[3]), "v"(s.m[4]), "v"(s.m[5]));
}
#undef MB_BCAST31
#undef MB_BCAST15
#undef MB_ROW
#undef MB_SCAN18
#undef MB_SCAN15

// Per-entry sums of the gradients gr[] of the evaluated queue positions
// [0, n): queued pairs of one entry are contiguous, a segmented scan over the
// lanes sums each entry's pairs and the segment's last lane writes (ADD =
// false) or adds to (ADD = true) the entry's slot. An entry that continues
// past position n - 1 (cont_j) leaves its partial sum in `carry`.
// The slot a segment's last lane adds to (pass 3), loaded before the pass's
// arithmetic so that the load's latency hides behind it; zero elsewhere.
struct SlotVals {
  float4 s[5];
};
__device__ __forceinline__ bool writes_slot(bool act, int j, int n, int lane, int cont_j) {
  const int jnext = __shfl_down(j, 1, 64);
  const bool last = act && (lane == n - 1 || jnext != j);
  return last && !(lane == n - 1 && j == cont_j);
}
__device__ __forceinline__ SlotVals load_slot(bool w, int j, const float* partials, const int* sk, int wave) {
  SlotVals v;  // read only by the lanes that load it
  if (w) {
    const float4* slot = reinterpret_cast<const float4*>(partials + ((size_t)sk[j] * 4 + wave) * kGradStride);
#pragma unroll
    for (int f = 0; f < 5; ++f) v.s[f] = slot[f];
  }
  return v;
}

// ADD = true adds the slot's earlier contents, passed in as `prev` (see
// load_slot); ADD = false overwrites the slot.
template <bool ADD>
__device__ __forceinline__ void reduce_to_slots(float* gr, bool act, int j, int n, int lane, int cont_j, int& carry_j,
                                                float* carry, float* partials, const int* sk, int wave,
                                                const SlotVals* prev = nullptr) {
  const int jprev = __shfl_up(j, 1, 64);
  const bool head = !act || lane == 0 || jprev != j;
  const uint64_t heads = __ballot(head);
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
  const int seg_start = 63 - __builtin_clzll(heads & upto);
  const int jnext = __shfl_down(j, 1, 64);
  const bool last = act && (lane == n - 1 || jnext != j);
  // the moment part (ADD) leaves the colour fields zero: they need no scan
  if constexpr (ADD)
    segment_scan15(gr, scan_masks(lane, seg_start));
  else
    segment_scan18(gr, scan_masks(lane, seg_start));
  if (last) {
    if (seg_start == 0 && j == carry_j) {
#pragma unroll
      for (int f = 0; f < G_COUNT; ++f) gr[f] += carry[f];
    }
    if (lane == n - 1 && j == cont_j) {
#pragma unroll
      for (int f = 0; f < G_COUNT; ++f) carry[f] = gr[f];
    } else {
      float4* slot = reinterpret_cast<float4*>(partials + ((size_t)sk[j] * 4 + wave) * kGradStride);
      if constexpr (ADD) {
        const float* pv = reinterpret_cast<const float*>(prev->s);
#pragma unroll
        for (int f = 0; f < G_COUNT; ++f) gr[f] += pv[f];
      }
      slot[0] = make_float4(gr[0], gr[1], gr[2], gr[3]);
      slot[1] = make_float4(gr[4], gr[5], gr[6], gr[7]);
      slot[2] = make_float4(gr[8], gr[9], gr[10], gr[11]);
      slot[3] = make_float4(gr[12], gr[13], gr[14], gr[15]);
      slot[4] = make_float4(gr[16], gr[17], 0.f, 0.f);
    }
  }
  __builtin_amdgcn_wave_barrier();
  // the entry continuing into the next evaluation (if any) owns the carry
  const int jl = __shfl(j, n - 1, 64);
  carry_j = (jl == cont_j) ? cont_j : -1;
}

// MODE 0: the moment bounds of Sec. 3.2 (power moments).
// MODE 1: the backward pass through the learned surrogate (the forward pass
// was mb_render_forward_surrogate): the optical depth at every edge is m_0 F
// with F and dF/d(inputs) from the query list, and the adjoint reaches the
// moments through the surrogate's inputs instead of the moment bounds.
// MODE 2: trigonometric moments (K = 4 or 6: two or three complex moments),
// the adjoint of the reconstruction on the circle (trig_adjoint) and of
// Eq. 14 (trig_moment_grads) in place of the power moments'.
template <int K, int NQ, int MODE>
__global__ __launch_bounds__(256, (K <= 6 && NQ == 4 && MODE == 0) ? 3 : 2) void k_render_bwd(BwdArgs ba,
                                                                                              CamSet cams) {
  constexpr bool SUR = MODE == 1;
  constexpr bool TRIG = MODE == 2;
  static_assert(!TRIG || K == 4 || K == 6, "the trigonometric path takes two or three complex moments");
  constexpr int NH = K / 2;
  constexpr int NL = (NH + 1) * (NH + 2) / 2;
  constexpr int RS = (K + 4) / 4 * 4;  // plain pass 2: K + 1 adjoint moments per pair, padded to float4s
  constexpr int NRES = SUR ? 9 : RS;   // results per queued pair ([k][64], or [64][RS] in the plain pass 2)
  const RenderArgs& a = ba.r;
  __shared__ Stage st;
  __shared__ int sk[kBlock];
  __shared__ WaveQueue wq[4];
  __shared__ uint32_t wrank[4][SUR ? 128 : 1];           // pair ranks (surrogate queries)
  __shared__ __align__(16) float wres[4][NRES * 64];     // per queued pair results
  __shared__ float carry[4][G_COUNT];                    // partial slot of an entry split over evaluations
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
  // as in the forward pass: a split block's waves share one quadrant and
  // take every fourth list entry; slots and masks are per (entry, quadrant)
  const bool split = bw.quad >= 0;
  const int quad = split ? bw.quad : wave;
  const int own4 = split ? wave : -1;
  const int x0 = tx * kTile + (quad & 1) * 8, y0 = ty * kTile + (quad >> 1) * 8;
  const int px = x0 + (lane & 7);
  const int py = y0 + (lane >> 3);
  const bool inside = px < c.width && py < c.height;
  const float u = (float)px + 0.5f, v = (float)py + 0.5f;
  const float rx = (u - c.cx) / c.fx, ry = (v - c.cy) / c.fy;
  const float lam = sqrtf(1.f + rx * rx + ry * ry);
  const float tn = c.tn;
  const int2 rg = a.ranges[key];
  const size_t pix = inside ? ((size_t)ci * c.height + py) * c.width + px : 0;
  WaveQueue& q = wq[wave];
  float* res = wres[wave];

  float sv[8] = {0.f, 0.f, 0.f, 0.f, tn + 1.f, 1.f, 0.f, 0.f};
  float gi[3] = {0.f, 0.f, 0.f};
  if (inside) {
    const float4* sp = reinterpret_cast<const float4*>(ba.saved + pix * MB_SAVED_FLOATS_PER_PIXEL);
    float4 s0 = sp[0], s1 = sp[1];
    sv[0] = s0.x; sv[1] = s0.y; sv[2] = s0.z; sv[3] = s0.w;
    sv[4] = s1.x; sv[5] = s1.y; sv[6] = s1.z; sv[7] = s1.w;
    gi[0] = ba.grad_image[pix * 3];
    gi[1] = ba.grad_image[pix * 3 + 1];
    gi[2] = ba.grad_image[pix * 3 + 2];
  }
  const bool want_gp = ba.grad_penalty != nullptr;
  const float gpen = (inside && want_gp) ? ba.grad_penalty[pix] : 0.f;
  const PixelBasis pb = make_basis(sv[4], sv[5], tn);

  auto basis_of = [&](int p) __attribute__((always_inline)) {
    PixelBasis r;
    r.tc = from_lane(pb.tc, p);
    r.p = from_lane(pb.p, p);
    r.p15 = from_lane(pb.p15, p);
    r.amp = from_lane(pb.amp, p);
    return r;
  };
  // the pair at queue position `lane` (entry j, pixel lane p); inactive lanes
  // (lane >= n) get p = lane so the cross-lane reads stay uniform
  auto item_of = [&](int n, int& j, int& p) __attribute__((always_inline)) {
    const bool act = lane < n;
    const int it = act ? (int)q.item[lane] : lane;
    j = act ? (it >> 6) : 0;
    p = it & 63;
    return act;
  };
  auto offsets_of = [&](int j, int p, float& dx, float& dy) __attribute__((always_inline)) {
    dx = (float)(x0 + (p & 7)) + 0.5f - st.f[0][j].x;
    dy = (float)(y0 + (p >> 3)) + 0.5f - st.f[0][j].y;
  };
  // flags: mark which of the entries' slots this block writes (an entry's
  // slot for a quadrant whose stored mask is empty is neither written nor
  // read: its sum is zero)
  auto stage = [&](int b, int nb, bool flags) __attribute__((always_inline)) {
    __syncthreads();
    load_batch_covered(st, a.rec, a.sorted_rec, a.masks, bw.quad, b, nb);
    if (tid < nb) {
      const int k = ba.sorted_k[b + tid];
      sk[tid] = k;
      if (flags) {
        const uint64_t* mp = a.masks + (size_t)(b + tid) * 4;
        if (bw.quad >= 0) {
          ba.used[(size_t)k * 4 + bw.quad] = mp[bw.quad] != 0ull ? 1 : 0;
        } else {
          uchar4 f;
          f.x = mp[0] != 0ull ? 1 : 0;
          f.y = mp[1] != 0ull ? 1 : 0;
          f.z = mp[2] != 0ull ? 1 : 0;
          f.w = mp[3] != 0ull ? 1 : 0;
          reinterpret_cast<uchar4*>(ba.used)[k] = f;
        }
      }
    }
    __syncthreads();
  };

  // ---- the pixel's moment sums, as the forward pass left them --------------
  double acc[K + 1];
#pragma unroll
  for (int k = 0; k <= K; ++k) acc[k] = inside ? a.pix_mom[(size_t)k * a.n_pix + pix] : 0.0;
  const float m0 = (float)acc[0];
  const bool live = acc[0] > kMinDepth;  // as in the forward pass
  LInv<NH> L;
  TrigLInv<TRIG ? NH : 1> TL;
  float bk[K + 1];
  bk[0] = 1.f;
  float mix_eps = 0.f;  // the forward pass's mixture weight (degenerate measures)
  if (live && !SUR) {
    double bn[K + 1], bmix[K + 1];
    bn[0] = 1.0;
#pragma unroll
    for (int k = 1; k <= K; ++k) {
      bn[k] = acc[k] / acc[0];
      bk[k] = (float)bn[k];
    }
    if constexpr (TRIG) {
      mix_eps = (float)trig_factor<NH>(acc, TL);
#pragma unroll
      for (int i = 0; i < NL; ++i) L.l[i] = 0.f;
    } else {
      mix_eps = (float)hankel_factor<NH>(bn, L, bmix);
    }
  } else {
    if constexpr (TRIG) {
#pragma unroll
      for (int i = 0; i < NL; ++i) TL.re[i] = TL.im[i] = 0.f;
    }
#pragma unroll
    for (int k = 1; k <= K; ++k) bk[k] = 0.f;
#pragma unroll
    for (int i = 0; i < NL; ++i) L.l[i] = 0.f;
  }

  // ---- Eq. 15 adjoint, folded into the two stages -------------------------
  const float alpha = -expm1f(-m0);
  const float oc = fmaxf(a.eps, sv[3]);
  float ga[3], gb, e0;
  {
    float gs = gi[0] * sv[0] + gi[1] * sv[1] + gi[2] * sv[2];
    float gbg = gi[0] * c.bg[0] + gi[1] * c.bg[1] + gi[2] * c.bg[2];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) ga[ch] = gi[ch] * alpha / oc;
    gb = sv[3] > a.eps ? -gs * alpha / (sv[3] * sv[3]) : 0.f;
    e0 = expf(-m0) * (gs / oc - gbg);
  }

  const bool active = inside && live;
  const uint64_t active_mask = __ballot(active);
  float* cw = carry[wave];
  // the slot of an entry whose stored mask has pixels, none of which this
  // pass keeps (outside the image, or without density), is written as zero
  auto zero_slot = [&](int j) __attribute__((always_inline)) {
    float4* slot = reinterpret_cast<float4*>(ba.partials + ((size_t)sk[j] * 4 + quad) * kGradStride);
#pragma unroll
    for (int f = 0; f < kGradStride / 4; ++f) slot[f] = make_float4(0.f, 0.f, 0.f, 0.f);
  };

  // ---- pass 2: adjoint moments, and the dm-independent gradients -----------
  float dm[K + 1];
#pragma unroll
  for (int k = 0; k <= K; ++k) dm[k] = 0.f;
  if constexpr (SUR) {
    static_assert(K == 6, "the surrogate takes six moments");
    // the forward pass's standardisation of the moment variable
    float smu = 0.f, ssig = 1.f;
    if (live) {
      const double mb = acc[1] / acc[0];
      const double var = acc[2] / acc[0] - mb * mb;
      smu = (float)mb;
      ssig = (float)(var > 0.0 ? sqrt(var) : 1.0);
    }
    // a pixel the forward pass left without queries (its list overflowed)
    // rendered as empty there and takes no gradient here
    const long long qb = active ? a.pix_qbase[pix] : -1;
    const uint64_t sur_mask = __ballot(qb >= 0);
    float dm0s = 0.f, dmus = 0.f, dsigs = 0.f, dfeat[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    QueueRanks rk{wrank[wave], 0u};
    int carry_j = -1;
    auto flush = [&](int n, uint64_t own, int cont_j) __attribute__((always_inline)) {
      int j, p;
      const bool act = item_of(n, j, p);
      const PixelBasis pp = basis_of(p);
      const float lamp = from_lane(lam, p), m0p = from_lane(m0, p);
      float gap[3] = {from_lane(ga[0], p), from_lane(ga[1], p), from_lane(ga[2], p)};
      const float gbp = from_lane(gb, p);
      const float smup = from_lane(smu, p), ssigp = from_lane(ssig, p);
      const uint32_t qlo = (uint32_t)__shfl((int)(uint32_t)(qb & 0xffffffffll), p, 64);
      const uint32_t qhi = (uint32_t)__shfl((int)(uint32_t)((unsigned long long)qb >> 32), p, 64);
      const long long qbase_p = (long long)(((unsigned long long)qhi << 32) | qlo);
      float gr[G_COUNT];
#pragma unroll
      for (int f = 0; f < G_COUNT; ++f) gr[f] = 0.f;
      if (act) {
        const uint32_t rank = wrank[wave][lane];
        float dx, dy;
        offsets_of(j, p, dx, dy);
        RayG g = ray_params(st, j, dx, dy, lamp);
        QuadState<NH, NQ> s;
        quad_geom<NH, NQ>(g, pp, tn, a, s);
        // F as the forward pass used it; its input gradient beside it
        const long long qi = qbase_p + (long long)rank * NQ;
        const float* qg = a.q_g + qi * 8;
        // the forward pass's running maximum: edge e takes the optical depth
        // of edge src[e] (the last edge at or before e that raised it)
        int src[NQ];
#pragma unroll
        for (int e = 0; e < NQ; ++e) {
          s.F[e] = a.q_f[qi + e];
          const float te = m0p * s.F[e];
          const bool up = e == 0 || te > s.tau[e > 0 ? e - 1 : 0];
          s.tau[e] = up ? te : s.tau[e > 0 ? e - 1 : 0];
          src[e] = up ? e : src[e > 0 ? e - 1 : 0];
        }
        quad_terms<NH, NQ>(g, tn, s);
        float4 f5 = st.f[5][j];
        const float gbar = gap[0] * f5.y + gap[1] * f5.z + gap[2] * f5.w + gbp;
        // dL/dtau gathered onto the edges whose queries supplied it
        float wsrc[NQ];
#pragma unroll
        for (int e = 0; e < NQ; ++e) wsrc[e] = 0.f;
#pragma unroll
        for (int e = 0; e < NQ; ++e) {
#pragma unroll
          for (int e2 = 0; e2 <= e; ++e2) wsrc[e2] += src[e] == e2 ? gbar * s.A[e] : 0.f;
        }
        float c[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        float gmu = 0.f, gsig = 0.f, gom = 0.f;
        const float isg = fast_rcp(ssigp);
#pragma unroll
        for (int e = 0; e < NQ; ++e) {
          const float* ge = qg + e * 8;
          const float wgt = wsrc[e];
          c[0] += wgt * s.F[e];  // tau = m_0 F at fixed inputs
#pragma unroll
          for (int k = 0; k < 6; ++k) c[1 + k] += wgt * m0p * ge[1 + k];
          const float zr = (s.y[e] - smup) / ssigp;
          const float gz = fabsf(zr) < 10.f ? wgt * m0p * ge[7] * isg : 0.f;  // dL/dy at the edge
          c[7] -= gz;       // z = (y - mu) / sig
          c[8] -= gz * zr;
          const float dydt = warp_dy(pp, s.t[e]);
          gmu += gz * dydt * (s.cl[e] ? 0.f : 1.f);
          gsig += gz * dydt * (s.cl[e] ? 0.f : a.kappa * a.xq[e]);
        }
        float dq0 = 0.f, dq1 = 0.f, dq2 = 0.f;
#pragma unroll
        for (int e = 0; e + 1 < NQ; ++e) {
          float cdt = s.T[e] * s.ph[e] * g.omega * s.sr[e];
          float dmu0 = s.cl[e] ? 0.f : 1.f, dmu1 = s.cl[e + 1] ? 0.f : 1.f;
          float dsg0 = s.cl[e] ? 0.f : a.kappa * a.xq[e], dsg1 = s.cl[e + 1] ? 0.f : a.kappa * a.xq[e + 1];
          dq0 += cdt * (dmu1 - dmu0);
          dq1 += cdt * (dsg1 - dsg0);
          float cs = s.T[e] * s.dt[e] * s.ph[e];
          if (s.cl[e]) {
            float r = (s.t[e] - g.mu) * fast_rcp(g.sig);
            float sj = g.omega * s.sr[e];
            const float igs = fast_rcp(g.sig);
            dq0 += cs * sj * r * igs;
            dq1 += cs * sj * r * r * igs;
          }
          dq2 += cs * s.sr[e];
        }
        gmu += gbar * dq0;
        gsig += gbar * dq1;
        gom += gbar * dq2;
#pragma unroll
        for (int k = 0; k < 9; ++k) res[k * 64 + lane] = c[k];
        chain_record(gmu, gsig, gom, g, lamp, dx, dy, st.f[2][j], st.f[3][j], st.f[4][j], gr);
        gr[G_CR] = s.q * gap[0];
        gr[G_CG] = s.q * gap[1];
        gr[G_CB] = s.q * gap[2];
      }
      __builtin_amdgcn_wave_barrier();
      while (own) {
        const int i = __builtin_ctzll(own);
        own &= own - 1;
        dm0s += res[i];
#pragma unroll
        for (int k = 0; k < 6; ++k) dfeat[k] += res[(1 + k) * 64 + i];
        dmus += res[7 * 64 + i];
        dsigs += res[8 * 64 + i];
      }
      reduce_to_slots<false>(gr, act, j, n, lane, cont_j, carry_j, cw, ba.partials, sk, quad);
    };
    for (int b = rg.x; b < rg.y; b += kBlock) {
      int nb = min(kBlock, rg.y - b);
      stage(b, nb, true);
      QueueCursor qc;
      queue_reset(qc);
      carry_j = -1;
      queue_from_masks(q, qc, a.masks, b, nb, quad, own4, lane, sur_mask,
                       [&]() __attribute__((always_inline)) {
                         const int cont_j = qc.cnt > 64 ? (int)(q.item[64] >> 6) : -1;
                         flush(64, qc.own_lo, cont_j);
                         queue_pop64<true>(q, qc, lane, wrank[wave]);
                       },
                       zero_slot, &rk);
      if (qc.cnt > 0) flush(qc.cnt, qc.own_lo, -1);
    }
    // the moment adjoint through the surrogate's inputs (forward-mode Jacobian
    // of the standardised features in double, one moment at a time)
    if (active) {
#pragma unroll 1
      for (int i = 0; i <= 6; ++i) {
        DualD md[7], feat[6], mu, sg;
#pragma unroll
        for (int k = 0; k <= 6; ++k) md[k] = DualD(acc[k], k == i ? 1.0 : 0.0);
        feat_from_moments(md, feat, mu, sg);
        double d = (i == 0 ? (double)dm0s : 0.0) + (double)dmus * mu.d + (double)dsigs * sg.d;
#pragma unroll
        for (int k = 0; k < 6; ++k) d += (double)dfeat[k] * feat[k].d;
        dm[i] = (float)d;
      }
      if (own4 <= 0) dm[0] += e0;
    }
  } else {
  dm[0] = (active && own4 <= 0) ? e0 : 0.f;  // a split block adds e0 once (wave 0)
  {
    int carry_j = -1;
    auto flush = [&](int n, uint64_t own, int cont_j) __attribute__((always_inline)) {
      int j, p;
      const bool act = item_of(n, j, p);
      const PixelBasis pp = basis_of(p);
      LInv<NH> Lp;
      TrigLInv<TRIG ? NH : 1> TLp;
      if constexpr (TRIG) {
#pragma unroll
        for (int i = 0; i < NL; ++i) {
          TLp.re[i] = from_lane(TL.re[i], p);
          TLp.im[i] = from_lane(TL.im[i], p);
        }
      } else {
#pragma unroll
        for (int i = 0; i < NL; ++i) Lp.l[i] = from_lane(L.l[i], p);
      }
      const float lamp = from_lane(lam, p), m0p = from_lane(m0, p);
      float gap[3] = {from_lane(ga[0], p), from_lane(ga[1], p), from_lane(ga[2], p)};
      const float gbp = from_lane(gb, p);
      const float gpp = from_lane(gpen, p);
      float bkp[K + 1];
      bkp[0] = 1.f;
#pragma unroll
      for (int k = 1; k <= K; ++k) bkp[k] = from_lane(bk[k], p);
      float gr[G_COUNT];
#pragma unroll
      for (int f = 0; f < G_COUNT; ++f) gr[f] = 0.f;
      if (act) {
        float dx, dy;
        offsets_of(j, p, dx, dy);
        RayG g = ray_params(st, j, dx, dy, lamp);
        QuadState<NH, NQ> s;
        TrigCanon<NH> tc[TRIG ? NQ : 1];
        int src[NQ];
        if constexpr (TRIG) {
          trig_quad_state<NH, NQ>(g, TLp, m0p, tn, a, s, tc, src);
        } else {
          quad_state<NH, NQ>(g, pp, Lp, m0p, tn, a, s);
        }
        float4 f5 = st.f[5][j];
        float gbar = gap[0] * f5.y + gap[1] * f5.z + gap[2] * f5.w + gbp;
        // consistency penalty (App. E): dP/dtau at the edges (bq, scaled by the
        // pixel's dL/dP) and its direct dependence on (mu, Sigma, omega)
        // through tau_ij = omega Sigma sqrt(pi/2) (erfc(b_j) - erfc(b_{j+1}))
        float bq[NQ];
#pragma unroll
        for (int e = 0; e < NQ; ++e) bq[e] = 0.f;
        float gmu = 0.f, gsig = 0.f, gom = 0.f;
        if (want_gp) {
          bool any_cl = false;
#pragma unroll
          for (int e = 0; e < NQ; ++e) any_cl = any_cl || s.cl[e];
          const float isg = fast_rcp(g.sig);
          const float bnear = (tn - g.mu) * kInvSqrt2 * isg;
          const float en = any_cl ? erfc_fast(bnear) : 0.f;
          const float gn = any_cl ? 1.1283791670955126f * __expf(-bnear * bnear) : 0.f;  // -d erfc / db
          const float cs = g.omega * g.sig * kSqrtHalfPi;
#pragma unroll
          for (int e = 0; e + 1 < NQ; ++e) {
            const float e0 = s.cl[e] ? en : a.ecq[e], e1 = s.cl[e + 1] ? en : a.ecq[e + 1];
            const float r = fmaxf(cs * (e0 - e1) - (s.tau[e + 1] - s.tau[e]), 0.f);
            const float tr = 2.f * r * gpp;
            bq[e] += tr;
            bq[e + 1] -= tr;
            const float ds0 = s.cl[e] ? gn * bnear * isg : 0.f, ds1 = s.cl[e + 1] ? gn * bnear * isg : 0.f;
            const float dm0 = s.cl[e] ? gn * kInvSqrt2 * isg : 0.f, dm1 = s.cl[e + 1] ? gn * kInvSqrt2 * isg : 0.f;
            gom += tr * g.sig * kSqrtHalfPi * (e0 - e1);
            gsig += tr * (g.omega * kSqrtHalfPi * (e0 - e1) + cs * (ds0 - ds1));
            gmu += tr * cs * (dm0 - dm1);
          }
        }
        float d[K + 1];
#pragma unroll
        for (int k = 0; k <= K; ++k) d[k] = 0.f;
        // (radiance + penalty) gradient at fixed moments: through tau at the
        // edges (which move with mu and Sigma) and the Eq. 7 interval terms
        if constexpr (TRIG) {
          // dL/dtau gathered onto the edges whose queries supplied it
          float wsrc[NQ];
#pragma unroll
          for (int e = 0; e < NQ; ++e) wsrc[e] = 0.f;
#pragma unroll
          for (int e = 0; e < NQ; ++e) {
#pragma unroll
            for (int e2 = 0; e2 <= e; ++e2) wsrc[e2] += src[e] == e2 ? gbar * s.A[e] + bq[e] : 0.f;
          }
#pragma unroll
          for (int e = 0; e < NQ; ++e) {
            float gk[K + 1], dpsi;
            trig_adjoint<NH>(s.y[e], tc[e], a.beta, gk, dpsi);
            const float wgt = wsrc[e];
#pragma unroll
            for (int k = 1; k <= K; ++k) d[k] += wgt * gk[k];
            d[0] += wgt * s.F[e];
            const float dtau_dt = m0p * dpsi * kTrigSpan * warp_abs_d(s.t[e], tn);
            gmu += wgt * dtau_dt * (s.cl[e] ? 0.f : 1.f);
            gsig += wgt * dtau_dt * (s.cl[e] ? 0.f : a.kappa * a.xq[e]);
          }
        } else {
#pragma unroll
          for (int e = 0; e < NQ; ++e) {
            float lamk[2 * NH + 1], dl;
            hermite_adjoint<NH>(s.y[e], s.x[e], s.below[e], a.beta, lamk, dl);
            float wgt = gbar * s.A[e] + bq[e];
#pragma unroll
            for (int k = 1; k <= K; ++k) d[k] += wgt * lamk[k];
            d[0] += wgt * s.F[e];  // minus sum_k b_k d[k], taken once after the edges
            float dtau_dt = -m0p * s.w0[e] * dl * warp_dy(pp, s.t[e]);
            float dtdmu = s.cl[e] ? 0.f : 1.f;
            float dtdsig = s.cl[e] ? 0.f : a.kappa * a.xq[e];
            gmu += wgt * dtau_dt * dtdmu;
            gsig += wgt * dtau_dt * dtdsig;
          }
        }
#pragma unroll
        for (int k = 1; k <= K; ++k) d[0] -= bkp[k] * d[k];  // the tau = m_0 F(b) chain at b = m / m_0
        float dq0 = 0.f, dq1 = 0.f, dq2 = 0.f;
#pragma unroll
        for (int e = 0; e + 1 < NQ; ++e) {
          float cdt = s.T[e] * s.ph[e] * g.omega * s.sr[e];
          float dmu0 = s.cl[e] ? 0.f : 1.f, dmu1 = s.cl[e + 1] ? 0.f : 1.f;
          float dsg0 = s.cl[e] ? 0.f : a.kappa * a.xq[e], dsg1 = s.cl[e + 1] ? 0.f : a.kappa * a.xq[e + 1];
          dq0 += cdt * (dmu1 - dmu0);
          dq1 += cdt * (dsg1 - dsg0);
          float cs = s.T[e] * s.dt[e] * s.ph[e];
          if (s.cl[e]) {
            float r = (s.t[e] - g.mu) * fast_rcp(g.sig);
            float sj = g.omega * s.sr[e];
            const float isg = fast_rcp(g.sig);
            dq0 += cs * sj * r * isg;
            dq1 += cs * sj * r * r * isg;
          }
          dq2 += cs * s.sr[e];
        }
        gmu += gbar * dq0;
        gsig += gbar * dq1;
        gom += gbar * dq2;
        float e[RS];
#pragma unroll
        for (int k = 0; k < RS; ++k) e[k] = k <= K ? d[k] : 0.f;
        float4* r4 = reinterpret_cast<float4*>(res + lane * RS);
#pragma unroll
        for (int q4 = 0; q4 < RS / 4; ++q4) r4[q4] = make_float4(e[4 * q4], e[4 * q4 + 1], e[4 * q4 + 2], e[4 * q4 + 3]);
        chain_record(gmu, gsig, gom, g, lamp, dx, dy, st.f[2][j], st.f[3][j], st.f[4][j], gr);
        gr[G_CR] = s.q * gap[0];
        gr[G_CG] = s.q * gap[1];
        gr[G_CB] = s.q * gap[2];
      }
      __builtin_amdgcn_wave_barrier();
      const float4* r4 = reinterpret_cast<const float4*>(res);
      struct Slots {
        float4 q[RS / 4];
      };
      for_each_own(
          own,
          [&](int i) __attribute__((always_inline)) {
            Slots v;
#pragma unroll
            for (int q4 = 0; q4 < RS / 4; ++q4) v.q[q4] = r4[i * (RS / 4) + q4];
            return v;
          },
          [&](const Slots& v) __attribute__((always_inline)) {
            const float* f = reinterpret_cast<const float*>(v.q);
#pragma unroll
            for (int k = 0; k <= K; ++k) dm[k] += f[k];
          });
      reduce_to_slots<false>(gr, act, j, n, lane, cont_j, carry_j, cw, ba.partials, sk, quad);
    };
    for (int b = rg.x; b < rg.y; b += kBlock) {
      int nb = min(kBlock, rg.y - b);
      stage(b, nb, true);
      QueueCursor qc;
      queue_reset(qc);
      carry_j = -1;
      queue_from_masks(q, qc, a.masks, b, nb, quad, own4, lane, active_mask,
                       [&]() __attribute__((always_inline)) {
                         const int cont_j = qc.cnt > 64 ? (int)(q.item[64] >> 6) : -1;
                         flush(64, qc.own_lo, cont_j);
                         queue_pop64(q, qc, lane);
                       },
                       zero_slot);
      if (qc.cnt > 0) flush(qc.cnt, qc.own_lo, -1);
    }
  }

  }
  if (split) {
    float* xf = reinterpret_cast<float*>(&st);
    __syncthreads();
#pragma unroll
    for (int k = 0; k <= K; ++k) xf[(wave * (K + 1) + k) * 64 + lane] = dm[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k <= K; ++k) {
      float t = 0.f;
#pragma unroll
      for (int w = 0; w < 4; ++w) t += xf[(w * (K + 1) + k) * 64 + lane];
      dm[k] = t;
    }
  }

  if (!SUR && active && mix_eps != 0.f) {
    // a degenerate pixel: the pairs took dL/db' at the mixture b' (dm[1..K]);
    // back to b through the mixture, and dm[0]'s share -sum_k b_k dL/db_k
    // follows the changed dL/db. With the identity factor F does not depend
    // on b, and the moments pass no gradient but m_0's.
    double bn[K + 1], D[K + 1];
    bn[0] = 1.0;
    D[0] = 0.0;
#pragma unroll
    for (int k = 1; k <= K; ++k) {
      bn[k] = (double)bk[k];
      D[k] = dm[k];
    }
    if (mix_eps > 0.f) {
      if constexpr (TRIG) {
        // mixed with the uniform measure on the circle: c' = (1 - eps) c + eps e_0
#pragma unroll
        for (int k = 1; k <= K; ++k) D[k] *= 1.0 - (double)mix_eps;
      } else {
        mixture_adjoint<K + 1>(bn, (double)mix_eps, D);
      }
    } else {
#pragma unroll
      for (int k = 1; k <= K; ++k) D[k] = 0.0;
    }
    double corr = 0.0;
#pragma unroll
    for (int k = 1; k <= K; ++k) corr += (double)bk[k] * ((double)dm[k] - D[k]);
    dm[0] += (float)corr;
#pragma unroll
    for (int k = 1; k <= K; ++k) dm[k] = (float)D[k];
  }

  // ---- pass 3: the moment part of the Gradient stage ------------------------
  {
    int carry_j = -1;
    auto flush = [&](int n, int cont_j) __attribute__((always_inline)) {
      int j, p;
      const bool act = item_of(n, j, p);
      const SlotVals prev = load_slot(writes_slot(act, j, n, lane, cont_j), j, ba.partials, sk, quad);
      const PixelBasis pp = basis_of(p);
      const float lamp = from_lane(lam, p);
      float dmp[K + 1];
#pragma unroll
      for (int k = 0; k <= K; ++k) dmp[k] = from_lane(dm[k], p);
      float gr[G_COUNT];
#pragma unroll
      for (int f = 0; f < G_COUNT; ++f) gr[f] = 0.f;
      if (act) {
        float dx, dy;
        offsets_of(j, p, dx, dy);
        RayG g = ray_params(st, j, dx, dy, lamp);
        float gm[3];
        if constexpr (TRIG)
          trig_moment_grads<NH>(g, tn, dmp, gm);
        else
          moment_grads<K>(g, pp, tn, dmp, gm);
        chain_record(gm[0], gm[1], gm[2], g, lamp, dx, dy, st.f[2][j], st.f[3][j], st.f[4][j], gr);
      }
      reduce_to_slots<true>(gr, act, j, n, lane, cont_j, carry_j, cw, ba.partials, sk, quad, &prev);
    };
    for (int b = rg.x; b < rg.y; b += kBlock) {
      int nb = min(kBlock, rg.y - b);
      stage(b, nb, false);
      QueueCursor qc;
      queue_reset(qc);
      carry_j = -1;
      queue_from_masks(q, qc, a.masks, b, nb, quad, own4, lane, active_mask,
                       [&]() __attribute__((always_inline)) {
                         const int cont_j = qc.cnt > 64 ? (int)(q.item[64] >> 6) : -1;
                         flush(64, cont_j);
                         queue_pop64(q, qc, lane);
                       },
                       [](int) {});
      if (qc.cnt > 0) flush(qc.cnt, -1);
    }
  }
}

hipError_t launch_render_backward(const RenderArgs& r, const float* saved, const float* grad_image,
                                  const float* grad_penalty, const int* sorted_k, float* partials,
                                  uint8_t* used, const CamSet& cams, int n_moments, int n_intervals,
                                  hipStream_t s, int mode) {
  BwdArgs ba{r, saved, grad_image, grad_penalty, sorted_k, partials, used};
  int n_keys = r.tiles_x * r.tiles_y * r.n_cams;
  dim3 grid(render_blocks(n_keys)), block(kBlock);
#define MB_LAUNCH(KK, NN, SS)                                                          \
  if (n_moments == KK && n_intervals == NN && mode == SS) {                            \
    hipLaunchKernelGGL((k_render_bwd<KK, NN + 1, SS>), grid, block, 0, s, ba, cams); \
    return hipGetLastError();                                                          \
  }
  MB_LAUNCH(4, 3, 0)
  MB_LAUNCH(6, 3, 0)
  MB_LAUNCH(4, 5, 0)
  MB_LAUNCH(6, 5, 0)
  MB_LAUNCH(8, 3, 0)
  MB_LAUNCH(8, 5, 0)
  MB_LAUNCH(6, 3, 1)
  MB_LAUNCH(6, 5, 1)
  MB_LAUNCH(4, 3, 2)
  MB_LAUNCH(4, 5, 2)
  MB_LAUNCH(6, 3, 2)
  MB_LAUNCH(6, 5, 2)
#undef MB_LAUNCH
  return hipErrorInvalidValue;
}

}  // namespace mb
