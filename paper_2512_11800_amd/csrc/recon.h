// Moment-bound reconstruction of the optical depth at a query (Sec. 3.2),
// per pixel and per query, in float32 registers.
//
// Per pixel the Hankel matrix H of the normalised moments b = m / m_0 is
// factored once (H = L L^T, in double) and L^-1 is kept. For a query y:
//   z = L^-1 v(y),  w_0 = 1 / |z|^2           (weight of the atom at y)
//   c = L^-T z = H^-1 v(y)                     (kernel polynomial K(x) = c . v(x))
//   x_i: the n real roots of K                 (other atoms)
//   w_i = 1 / |L^-1 v(x_i)|^2                  (Christoffel numbers; equal to
//                                               the Vandermonde solve)
//   F = sum_{x_i < y} w_i + beta w_0           (= (1-beta) L + beta U, normalised)
// and the optical depth is m_0 F.
#pragma once
#include "common.h"

namespace mb {

template <int NH>
struct LInv {
  float l[(NH + 1) * (NH + 2) / 2];  // rows of lower-triangular L^-1, packed
};

// L^-1 v(x) for v(x) = (1, x, .., x^NH)
template <int NH>
__device__ __forceinline__ void linv_apply(const LInv<NH>& L, float x, float* z) {
  float p[NH + 1];
  p[0] = 1.f;
#pragma unroll
  for (int k = 1; k <= NH; ++k) p[k] = p[k - 1] * x;
  int o = 0;
#pragma unroll
  for (int i = 0; i <= NH; ++i) {
    float s = L.l[o];  // p[0] = 1; the sums start from their first term (no 0 + x)
#pragma unroll
    for (int j = 1; j <= i; ++j) s = fmaf(L.l[o + j], p[j], s);
    z[i] = s;
    o += i + 1;
  }
}

template <int NH>
__device__ __forceinline__ float christoffel(const LInv<NH>& L, float x) {
  float z[NH + 1];
  linv_apply<NH>(L, x, z);
  float s = z[0] * z[0];
#pragma unroll
  for (int i = 1; i <= NH; ++i) s = fmaf(z[i], z[i], s);
  return fast_rcp(s);
}

// c = L^-T z
template <int NH>
__device__ __forceinline__ void linv_t_apply(const LInv<NH>& L, const float* z, float* c) {
  // c_j = sum_{i >= j} L[i][j] z_i, from the last row up (row i starts at i (i + 1) / 2)
#pragma unroll
  for (int j = 0; j <= NH; ++j) c[j] = L.l[NH * (NH + 1) / 2 + j] * z[NH];
#pragma unroll
  for (int i = NH - 1; i >= 0; --i) {
#pragma unroll
    for (int j = 0; j <= i; ++j) c[j] = fmaf(L.l[i * (i + 1) / 2 + j], z[i], c[j]);
  }
}

// Real roots of c0 + c1 x + c2 x^2 (stable form).
__device__ __forceinline__ void roots2(const float* c, float* x) {
  float disc = fmaxf(c[1] * c[1] - 4.f * c[2] * c[0], 0.f);
  float sq = fast_sqrt(disc);
  float q = -0.5f * (c[1] + copysignf(sq, c[1]));
  x[0] = q * fast_rcp(c[2]);
  x[1] = c[0] * fast_rcp(q);
}

__device__ __forceinline__ float cubic_newton(const float* c, float x, int iters) {
  for (int it = 0; it < iters; ++it) {
    float p = ((c[3] * x + c[2]) * x + c[1]) * x + c[0];
    float dp = (3.f * c[3] * x + 2.f * c[2]) * x + c[1];
    float st = p * fast_rcp(dp);
    x = (dp != 0.f && isfinite(st)) ? x - st : x;
  }
  return x;
}

// Real roots of c0 + c1 x + c2 x^2 + c3 x^3 (three real roots for a positive
// definite Hankel matrix). The trigonometric solution is accurate only for the
// root of largest magnitude when the roots span a wide range (c3 -> 0 sends
// one atom of the canonical representation to infinity), so that root is
// taken from it, polished, divided out from the low-order end (stable for a
// large root) and the remaining quadratic is solved in its stable form; all
// roots get Newton steps on the full cubic.
__device__ __forceinline__ void roots3(const float* c, float* x) {
  float scale = fabsf(c[0]) + fabsf(c[1]) + fabsf(c[2]) + fabsf(c[3]);
  if (!(fabsf(c[3]) > 1e-12f * scale)) {
    // degree drop: one atom at infinity (zero weight)
    roots2(c, x);
    x[2] = copysignf(1e30f, -c[2] * c[3]);
    return;
  }
  float inv = fast_rcp(c[3]);
  float a = c[2] * inv, b = c[1] * inv, cc = c[0] * inv;
  float a3 = a * (1.f / 3.f);
  float q = a3 * a3 - b * (1.f / 3.f);
  float r = a3 * a3 * a3 - 0.5f * a3 * b + 0.5f * cc;
  q = fmaxf(q, 0.f);
  float sq = fast_sqrt(q);
  float den = q * sq;
  float arg = den > 0.f ? fminf(fmaxf(r * fast_rcp(den), -1.f), 1.f) : 0.f;
  // the trigonometric roots only seed the Newton steps below, so a short
  // arccosine (Abramowitz & Stegun 4.4.45, |error| < 7e-5) and the hardware
  // cosine are accurate enough
  const float aa = fabsf(arg);
  float ac = fast_sqrt(1.f - aa) * (1.5707288f + aa * (-0.2121144f + aa * (0.0742610f + aa * -0.0187293f)));
  ac = arg < 0.f ? 3.14159265358979f - ac : ac;
  float th = ac * (1.f / 3.f);
  const float two_pi_3 = 2.0943951023931953f;
  float big = 0.f;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    float xk = -2.f * sq * __cosf(th + two_pi_3 * (float)k) - a3;
    big = fabsf(xk) > fabsf(big) ? xk : big;
  }
  big = cubic_newton(c, big, 2);
  // p(x) = (x - big)(A x^2 + B x + C), matched from the constant term up
  float ib = fast_rcp(big);
  float cq = -c[0] * ib;
  float bq = (cq - c[1]) * ib;
  float aq = (bq - c[2]) * ib;
  float qc[3] = {cq, bq, aq};
  float x2[2];
  roots2(qc, x2);
  x[0] = big;
  x[1] = cubic_newton(c, x2[0], 2);
  x[2] = cubic_newton(c, x2[1], 2);
}

__device__ __forceinline__ float quartic_newton(const float* c, float x, int iters) {
  for (int it = 0; it < iters; ++it) {
    float p = (((c[4] * x + c[3]) * x + c[2]) * x + c[1]) * x + c[0];
    float dp = ((4.f * c[4] * x + 3.f * c[3]) * x + 2.f * c[2]) * x + c[1];
    float st = p * fast_rcp(dp);
    x = (dp != 0.f && isfinite(st)) ? x - st : x;
  }
  return x;
}

// Laguerre's iteration on the monic quartic x^4 + a3 x^3 + a2 x^2 + a1 x + a0.
// Started just outside the roots of a polynomial whose roots are all real,
// it moves monotonically to the nearest (extreme) root.
__device__ __forceinline__ float laguerre4(const float* a, float x, int iters) {
  for (int it = 0; it < iters; ++it) {
    float p = (((x + a[3]) * x + a[2]) * x + a[1]) * x + a[0];
    float d1 = ((4.f * x + 3.f * a[3]) * x + 2.f * a[2]) * x + a[1];
    float d2 = (12.f * x + 6.f * a[3]) * x + 2.f * a[2];
    float ip = fast_rcp(p);
    float g = d1 * ip;
    float h = g * g - d2 * ip;
    float sq = fast_sqrt(fmaxf(3.f * (4.f * h - g * g), 0.f));
    float den = g >= 0.f ? g + sq : g - sq;
    float st = 4.f * fast_rcp(den);
    x = (p != 0.f && den != 0.f && isfinite(st)) ? x - st : x;
  }
  return x;
}

// Real roots of c0 + c1 x + .. + c4 x^4 (four real roots for a positive
// definite Hankel matrix). By Samuelson's inequality every root lies within
// mean +- sqrt(3) sd of the roots (both read off the two leading
// coefficients); Laguerre's iteration from just outside that interval on
// either side gives the two extreme roots. The one of larger magnitude is
// divided out from the low-order end (stable for the dominant root), the
// cubic left over goes to roots3, and every root gets Newton steps on the
// full quartic. A vanishing leading coefficient sends one atom to infinity.
__device__ __forceinline__ void roots4(const float* c, float* x) {
  float scale = fabsf(c[0]) + fabsf(c[1]) + fabsf(c[2]) + fabsf(c[3]) + fabsf(c[4]);
  if (!(fabsf(c[4]) > 1e-12f * scale)) {
    roots3(c, x);
    x[3] = copysignf(1e30f, -c[3] * c[4]);
    return;
  }
  float inv = fast_rcp(c[4]);
  float a[4] = {c[0] * inv, c[1] * inv, c[2] * inv, c[3] * inv};
  float mean = -0.25f * a[3];
  float var = fmaxf(0.25f * (a[3] * a[3] - 2.f * a[2]) - mean * mean, 0.f);
  float half = fast_sqrt(3.f * var) * 1.0001f + 1e-6f * (fabsf(mean) + 1.f);
  float hi = laguerre4(a, mean + half, 4);
  float lo = laguerre4(a, mean - half, 4);
  float big = quartic_newton(c, fabsf(hi) >= fabsf(lo) ? hi : lo, 1);
  // p(x) = (x - big)(A x^3 + B x^2 + C x + D), matched from the constant term up
  float ib = fast_rcp(big);
  float d = -c[0] * ib;
  float cc = (d - c[1]) * ib;
  float b = (cc - c[2]) * ib;
  float aa = (b - c[3]) * ib;
  float qc[4] = {d, cc, b, aa};
  float x3[3];
  roots3(qc, x3);
  x[0] = big;
#pragma unroll
  for (int i = 0; i < 3; ++i) x[i + 1] = quartic_newton(c, x3[i], 2);
}

template <int NH>
__device__ __forceinline__ void kernel_roots(const float* c, float* x) {
  static_assert(NH >= 2 && NH <= 4, "two to four atoms besides the query");
  if constexpr (NH == 2)
    roots2(c, x);
  else if constexpr (NH == 3)
    roots3(c, x);
  else
    roots4(c, x);
}

// sum_{x_i < y} w_i from the count of atoms below y: the weights of the
// canonical representation sum to b_0 = 1, so with c of the NH atoms below,
// the sum is 0 (c = 0), 1 - w_0 (c = NH), and otherwise the Christoffel
// weights of the smaller side: the atoms below when c <= NH / 2, else 1 - w_0
// less the atoms above. At most one weight is evaluated for NH <= 3 and two
// for NH = 4. A root that is not a number counts as an atom above
// everything with no weight.
template <int NH>
__device__ __forceinline__ float mass_below(const LInv<NH>& L, float y, float w0, float* x) {
  int cnt = 0;
#pragma unroll
  for (int i = 0; i < NH; ++i) {
    x[i] = x[i] == x[i] ? x[i] : 1e30f;
    cnt += x[i] < y ? 1 : 0;
  }
  auto weight = [&](float xs) __attribute__((always_inline)) {
    const float w = christoffel<NH>(L, xs);
    return isfinite(w) ? w : 0.f;
  };
  if constexpr (NH == 2) {
    const float ws = weight(x[0] < y ? x[0] : x[1]);
    return cnt == 1 ? ws : (cnt == 2 ? 1.f - w0 : 0.f);
  } else if constexpr (NH == 3) {
    const float lo = fminf(fminf(x[0], x[1]), x[2]);
    const float hi = fmaxf(fmaxf(x[0], x[1]), x[2]);
    const float ws = weight(cnt <= 1 ? lo : hi);
    return cnt == 0 ? 0.f : (cnt == 1 ? ws : (cnt == 2 ? 1.f - w0 - ws : 1.f - w0));
  } else {
    // sorting network: s0 <= s1 <= s2 <= s3
    float s0 = fminf(x[0], x[1]), s1 = fmaxf(x[0], x[1]);
    float s2 = fminf(x[2], x[3]), s3 = fmaxf(x[2], x[3]);
    float t = fminf(s0, s2);
    s2 = fmaxf(s0, s2);
    s0 = t;
    t = fmaxf(s1, s3);
    s1 = fminf(s1, s3);
    s3 = t;
    t = fminf(s1, s2);
    s2 = fmaxf(s1, s2);
    s1 = t;
    const float wa = weight(cnt <= 2 ? s0 : s3);
    const float wb = weight(s1);
    return cnt == 0 ? 0.f
                    : (cnt == 1 ? wa : (cnt == 2 ? wa + wb : (cnt == 3 ? 1.f - w0 - wa : 1.f - w0)));
  }
}

// Normalised interpolated bound F(y) = sum_{x_i<y} w_i + beta w_0.
template <int NH>
__device__ __forceinline__ float bound_F(const LInv<NH>& L, float y, float beta) {
  float z[NH + 1], c[NH + 1], x[NH];
  linv_apply<NH>(L, y, z);
  float zz = z[0] * z[0];
#pragma unroll
  for (int i = 1; i <= NH; ++i) zz = fmaf(z[i], z[i], zz);
  const float w0 = fast_rcp(zz);
  linv_t_apply<NH>(L, z, c);
  kernel_roots<NH>(c, x);
  return mass_below<NH>(L, y, w0, x) + beta * w0;
}

// Canonical representation at y with its atoms (for the adjoint): returns F
// and fills the other atoms x_i, the flags x_i < y and the weight w_0 at y.
template <int NH>
__device__ __forceinline__ float canon_at(const LInv<NH>& L, float y, float beta, float* x, bool* below,
                                          float& w0) {
  float z[NH + 1], c[NH + 1];
  linv_apply<NH>(L, y, z);
  float zz = z[0] * z[0];
#pragma unroll
  for (int i = 1; i <= NH; ++i) zz = fmaf(z[i], z[i], zz);
  w0 = fast_rcp(zz);
  linv_t_apply<NH>(L, z, c);
  kernel_roots<NH>(c, x);
  const float lo = mass_below<NH>(L, y, w0, x);
#pragma unroll
  for (int i = 0; i < NH; ++i) below[i] = x[i] < y;
  return lo + beta * w0;
}

// Adjoint of F(y; b) = sum_{x_i < y} w_i + beta w_0 through the moment
// equations sum_i w_i x_i^k = b_k (k = 0..2n, x_0 = y): the polynomial
// Lambda of degree 2n with Lambda(x_i) = [x_i < y], Lambda'(x_i) = 0 (i >= 1)
// and Lambda(y) = beta has coefficients dF/db_k, and dF/dy = -w_0 Lambda'(y).
// Built by Hermite interpolation, then expanded to monomial coefficients.
// NH = 2 in closed form: Lambda = A + C P with A the cubic Hermite
// interpolant of the two atoms with zero slopes, A(x) = f1 + (f2 - f1)
// S((x - x1) / (x2 - x1)), S(t) = 3 t^2 - 2 t^3, P(x) = (x - x1)^2 (x - x2)^2
// and C = (beta - A(y)) / P(y), expanded to monomial coefficients.
__device__ __forceinline__ void hermite_adjoint2(float y, const float* xs, const bool* below, float beta,
                                                 float* lam, float& dlam_y) {
  const float x1 = fminf(fmaxf(xs[0], -1e6f), 1e6f), x2 = fminf(fmaxf(xs[1], -1e6f), 1e6f);
  const float f1 = below[0] ? 1.f : 0.f, f2 = below[1] ? 1.f : 0.f;
  const float D = f2 - f1;  // nonzero only for distinct atoms on either side of y
  const float h = x2 - x1;
  const float r = (D != 0.f && h != 0.f) ? fast_rcp(h) : 0.f;
  const float Dr2 = D * r * r, Dr3 = Dr2 * r;
  // A(x) = f1 + 3 D r^2 (x - x1)^2 - 2 D r^3 (x - x1)^3
  const float a3 = -2.f * Dr3;
  const float a2 = 3.f * Dr2 + 6.f * Dr3 * x1;
  const float a1 = -6.f * x1 * (Dr2 + Dr3 * x1);
  const float a0 = f1 + x1 * x1 * (3.f * Dr2 + 2.f * Dr3 * x1);
  const float uy = y - x1, vy = y - x2;
  const float ay = f1 + uy * uy * (3.f * Dr2 - 2.f * Dr3 * uy);
  const float sq = uy * vy;
  const float py = sq * sq;
  const float C = py != 0.f ? (beta - ay) * fast_rcp(py) : 0.f;
  // P(x) = x^4 - 2 s x^3 + (s^2 + 2 p) x^2 - 2 s p x + p^2
  const float sm = x1 + x2, pr = x1 * x2;
  lam[4] = C;
  lam[3] = a3 - 2.f * sm * C;
  lam[2] = a2 + (sm * sm + 2.f * pr) * C;
  lam[1] = a1 - 2.f * sm * pr * C;
  lam[0] = a0 + pr * pr * C;
  dlam_y = ((4.f * lam[4] * y + 3.f * lam[3]) * y + 2.f * lam[2]) * y + lam[1];
}

// Any NH: Newton divided differences on the nodes x_1, x_1, .., x_n, x_n, y.
template <int NH>
__device__ __forceinline__ void hermite_adjoint_dd(float y, const float* xs, const bool* below, float beta,
                                                   float* lam, float& dlam_y) {
  constexpr int NN = 2 * NH + 1;
  float z[NN], f[NN], coef[NN];
#pragma unroll
  for (int i = 0; i < NH; ++i) {
    // atoms sent towards infinity carry no weight; keep the arithmetic finite
    float xi = fminf(fmaxf(xs[i], -1e6f), 1e6f);
    z[2 * i] = xi;
    z[2 * i + 1] = xi;
    f[2 * i] = below[i] ? 1.f : 0.f;
    f[2 * i + 1] = f[2 * i];
  }
  z[NN - 1] = y;
  f[NN - 1] = beta;
  coef[0] = f[0];
#pragma unroll
  for (int order = 1; order < NN; ++order) {
#pragma unroll
    for (int a = 0; a + order < NN; ++a) {
      float dz = z[a + order] - z[a];
      f[a] = dz != 0.f ? (f[a + 1] - f[a]) * fast_rcp(dz) : 0.f;  // equal nodes: zero slope
    }
    coef[order] = f[0];
  }
  // Newton form -> monomial coefficients
  float p[NN];
#pragma unroll
  for (int k = 0; k < NN; ++k) p[k] = 0.f;
  p[0] = coef[NN - 1];
#pragma unroll
  for (int k = NN - 2; k >= 0; --k) {
    const int deg = NN - 2 - k;  // degree of p before multiplying by (x - z_k)
    p[deg + 1] = p[deg];
#pragma unroll
    for (int d = deg; d >= 1; --d) p[d] = p[d - 1] - z[k] * p[d];
    p[0] = coef[k] - z[k] * p[0];
  }
  float dl = 0.f;
#pragma unroll
  for (int k = NN - 1; k >= 1; --k) dl = dl * y + (float)k * p[k];
#pragma unroll
  for (int k = 0; k < NN; ++k) lam[k] = p[k];
  dlam_y = dl;
}

template <int NH>
__device__ __forceinline__ void hermite_adjoint(float y, const float* xs, const bool* below, float beta,
                                                float* lam, float& dlam_y) {
  if constexpr (NH == 2)
    hermite_adjoint2(y, xs, below, beta, lam, dlam_y);
  else
    hermite_adjoint_dd<NH>(y, xs, below, beta, lam, dlam_y);
}

// ---------------------------------------------------------------------------
// Per-pixel set-up of the bounds: the Cholesky factor of the Hankel matrix of
// the normalised moments b (b_0 = 1), kept as L^-1 in float.
//
// Degenerate measures. A ray density is a sum of Gaussians, so its Hankel
// matrices are positive definite in exact arithmetic; a measure that is
// nearly atomic (ray Gaussians far thinner than their separation) is singular
// to working precision. The test is taken on the standardised moments
// c_k = E[((y - mean) / sd)^k], which do not depend on the affine moment
// variable: the measure is degenerate when a Cholesky pivot of their Hankel
// matrix falls below kPivotRel times its diagonal entry (1e-5: a hundred times
// the float32 rounding the per-pair moments carry into these pivots, so the
// decision does not hinge on rounding). A degenerate measure
// is replaced by its mixture (1 - eps) mu + eps N(mean, sd^2) with the normal
// distribution of its own mean and variance, for the first eps of
// kMixEps[] that passes the test (the smallest, 1e-3, keeps the mixture's
// Hankel matrix conditioned to about 1e3, so its bounds and their adjoint
// stay accurate in float). The mixture is a valid measure with a
// positive definite Hankel matrix, it transforms with the moment variable, and
// it is differentiable in b (the backward pass applies its Jacobian). A moment
// vector without a positive variance or with non-finite entries gets the
// identity factor (finite, meaningless bounds). Both outcomes are flagged.
// ---------------------------------------------------------------------------
constexpr double kPivotRel = 1e-5;
constexpr int kMixLevels = 4;
__device__ constexpr double kMixEps[kMixLevels] = {1e-3, 1e-2, 1e-1, 1.0};

// Cholesky of the Hankel matrix of c (c_0 = 1): every pivot above kPivotRel
// times its diagonal entry, and the factor in lc when so.
template <int M>
__device__ __forceinline__ bool hankel_chol(const double* c, double (&lc)[M][M]) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    double s = c[2 * j];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= lc[j][k] * lc[j][k];
    ok = ok && (s > kPivotRel * c[2 * j]);
    const double d = sqrt(fmax(s, 1e-300));
    lc[j][j] = d;
#pragma unroll
    for (int i = j + 1; i < M; ++i) {
      double t = c[i + j];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= lc[i][k] * lc[j][k];
      lc[i][j] = t / d;
    }
  }
  return ok;
}

// moments E[(m + sd Z)^k], k = 0..2n, of N(m, v): n_k = m n_{k-1} + (k - 1) v n_{k-2}
template <int NK>
__device__ __forceinline__ void normal_moments(double m, double v, double* nm) {
  nm[0] = 1.0;
  nm[1] = m;
#pragma unroll
  for (int k = 2; k < NK; ++k) nm[k] = m * nm[k - 1] + (double)(k - 1) * v * nm[k - 2];
}

// Returns the mixture weight eps used (0: none; -1: identity factor) and the
// moments the factor belongs to in bmix[0..2 NH].
template <int NH>
__device__ __forceinline__ double hankel_factor(const double* b, LInv<NH>& out, double* bmix) {
  constexpr int M = NH + 1;
  constexpr int NK = 2 * NH + 1;
  const double mean = b[1], var = b[2] - b[1] * b[1];
  bool finite = true;
#pragma unroll
  for (int k = 0; k < NK; ++k) finite = finite && isfinite(b[k]);
  double eps = -1.0;
  if (finite && var > 0.0) {
    // standardised moments c_k = sum_j C(k, j) b_j (-mean)^(k - j) / sd^k
    const double is = 1.0 / sqrt(var);
    double c[NK], sn[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      double acc = 0.0, binom = 1.0, pw = 1.0;
#pragma unroll
      for (int j = k; j >= 0; --j) {
        acc += binom * b[j] * pw;
        binom = binom * (double)j / (double)(k - j + 1);
        pw *= -mean;
      }
      double sk = 1.0;
#pragma unroll
      for (int i = 0; i < k; ++i) sk *= is;
      c[k] = acc * sk;
    }
    normal_moments<NK>(0.0, 1.0, sn);
    double lc[M][M];
    if (hankel_chol<M>(c, lc)) {
      eps = 0.0;
    } else {
#pragma unroll 1
      for (int l = 0; l < kMixLevels && eps < 0.0; ++l) {
        double cm[NK];
#pragma unroll
        for (int k = 0; k < NK; ++k) cm[k] = (1.0 - kMixEps[l]) * c[k] + kMixEps[l] * sn[k];
        if (hankel_chol<M>(cm, lc)) eps = kMixEps[l];
      }
    }
  }
  double nm[NK];
  normal_moments<NK>(mean, var, nm);
#pragma unroll
  for (int k = 0; k < NK; ++k) bmix[k] = eps > 0.0 ? (1.0 - eps) * b[k] + eps * nm[k] : b[k];
  // the factor in the pixel's moment variable
  double lc[M][M];
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = 0; j < M; ++j) lc[i][j] = 0.0;
  bool ok = eps >= 0.0;
  if (ok) {
#pragma unroll
    for (int j = 0; j < M; ++j) {
      double s = bmix[2 * j];
#pragma unroll
      for (int k = 0; k < j; ++k) s -= lc[j][k] * lc[j][k];
      ok = ok && s > 0.0;
      const double d = sqrt(fmax(s, 1e-300));
      lc[j][j] = d;
#pragma unroll
      for (int i = j + 1; i < M; ++i) {
        double t = bmix[i + j];
#pragma unroll
        for (int k = 0; k < j; ++k) t -= lc[i][k] * lc[j][k];
        lc[i][j] = t / d;
      }
    }
  }
  if (!ok) {
    // no positive definite matrix: keep the arithmetic finite with the identity
    eps = -1.0;
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
      for (int j = 0; j < M; ++j) lc[i][j] = i == j ? 1.0 : 0.0;
  }
  // invert the lower-triangular factor
  double li[M][M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
#pragma unroll
    for (int j = 0; j < M; ++j) li[i][j] = 0.0;
    li[i][i] = 1.0 / lc[i][i];
#pragma unroll
    for (int j = 0; j < i; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = j; k < i; ++k) s += lc[i][k] * li[k][j];
      li[i][j] = -s / lc[i][i];
    }
  }
  int o = 0;
#pragma unroll
  for (int i = 0; i < M; ++i) {
#pragma unroll
    for (int j = 0; j <= i; ++j) out.l[o + j] = (float)li[i][j];
    o += i + 1;
  }
  return eps;
}

// Adjoint of the mixture b' = (1 - eps) b + eps n(b_1, b_2 - b_1^2) (n: the
// normal moments above) for k = 1..2n: given D = dL/db' (D[0] unused),
// returns dL/db in D. dn_k/dmean = k n_{k-1}, dn_k/dvar = k (k - 1) / 2 n_{k-2}.
template <int NK>
__device__ __forceinline__ void mixture_adjoint(const double* b, double eps, double* D) {
  const double mean = b[1], var = b[2] - b[1] * b[1];
  double nm[NK];
  normal_moments<NK>(mean, var, nm);
  double gm = 0.0, gv = 0.0;
#pragma unroll
  for (int k = 1; k < NK; ++k) {
    gm += D[k] * (double)k * nm[k - 1];
    if (k >= 2) gv += D[k] * 0.5 * (double)(k * (k - 1)) * nm[k - 2];
  }
#pragma unroll
  for (int k = 1; k < NK; ++k) D[k] *= 1.0 - eps;
  // mean = b_1, var = b_2 - b_1^2
  D[1] += eps * (gm - 2.0 * mean * gv);
  D[2] += eps * gv;
}

}  // namespace mb
