// Trigonometric moments of the ray density (Sec. 3.2, Eqs. 13-14, App. C)
// and the reconstruction of the optical depth from them on the circle.
//
// The warped depth g_hat(t) in [0, 1) is placed on the unit circle at the
// angle phi = (2 pi - theta) g_hat; the arc (2 pi - theta, 2 pi) stays empty
// (the wrapping zone; theta = 0.2 pi). The moments are the Fourier
// coefficients c_k = sum_j int e^{i k phi(t)} sigma_j(t) dt, k = 0..n, stored
// per pixel as (c_0, Re c_1, Im c_1, .., Re c_n, Im c_n): the 2n + 1 = K + 1
// reals a K-moment power basis stores.
//
// Reconstruction at a query angle psi, w = e^{i psi}: the canonical
// representation through w (the Gauss-Szego quadrature of the Toeplitz
// matrix T_jk = c_{k-j} of c / c_0). With T = L L^H (kept as L^-1):
//   u = L^-1 conj(v(w)),  lambda_0 = 1 / |u|^2       (weight of the atom at w)
//   a = L^-H u = T^-1 conj(v(w))                     (q(z) = sum_k a_k z^k)
//   z_i: the n zeros of q, on the unit circle       (other atoms)
//   lambda_i = 1 / |L^-1 conj(v(z_i))|^2             (Christoffel numbers)
// The atoms are ordered along the circle cut in the middle of the wrapping
// zone; F = sum_{atoms before w} lambda_i + beta lambda_0 and the optical
// depth is c_0 F. Along a Gaussian's edges it is made non-decreasing (the
// circle's estimates need not grow with depth).
#pragma once
#include "render_common.h"

namespace mb {

constexpr float kTrigSpan = 5.654866776461628f;  // 2 pi - theta, theta = 0.2 pi

struct cfl {
  float re, im;
};
__device__ __forceinline__ cfl cmul(cfl a, cfl b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cfl cadd(cfl a, cfl b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cfl csub(cfl a, cfl b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cfl cconj(cfl a) { return {a.re, -a.im}; }
__device__ __forceinline__ float cabs2(cfl a) { return a.re * a.re + a.im * a.im; }
__device__ __forceinline__ cfl cdiv(cfl a, cfl b) {
  const float s = fast_rcp(cabs2(b));
  return {(a.re * b.re + a.im * b.im) * s, (a.im * b.re - a.re * b.im) * s};
}
// principal square root
__device__ __forceinline__ cfl csqrt(cfl a) {
  const float r = sqrtf(cabs2(a));
  if (a.re >= 0.f) {
    const float re = sqrtf(0.5f * (r + a.re));
    return {re, re > 0.f ? 0.5f * a.im / re : 0.f};
  }
  const float im = copysignf(sqrtf(0.5f * (r - a.re)), a.im);
  return {0.5f * a.im / im, im};
}

template <int NH>
struct TrigLInv {
  float re[(NH + 1) * (NH + 2) / 2], im[(NH + 1) * (NH + 2) / 2];  // rows of L^-1, packed
};

// g_hat(t) itself (not the pixel's moment variable): 1 - ((1 + 0.8 t) / (1 + 0.8 t_n))^-1.5
__device__ __forceinline__ float warp_abs(float t, float tn) {
  const float r = (1.f + 0.8f * tn) * fast_rcp(1.f + 0.8f * t);
  return 1.f - r * fast_sqrt(r);
}
__device__ __forceinline__ float warp_abs_d(float t, float tn) {  // d g_hat / dt = 1.2 r^1.5 / (1 + 0.8 t)
  const float q = 1.f + 0.8f * t;
  const float r = (1.f + 0.8f * tn) * fast_rcp(q);
  return 1.2f * r * fast_sqrt(r) * fast_rcp(q);
}

// Eq. 14 for one ray Gaussian, k = 0..NH, with the first-order complex erf of
// App. C: c_k = A D^(k^2) z^k (erfc(a) + i k b (2 / sqrt pi) e^{-a^2}), where
// A = omega Sigma sqrt(pi / 2), z = e^{i alpha_1 G}, D = e^{-Sigma^2 alpha_1^2 G'^2 / 2},
// b = Sigma alpha_1 G' / sqrt 2, a = (t_n - mu) / (sqrt2 Sigma). The phase
// alpha_1 G, its sine and cosine, and the damping D are evaluated in double
// from the float ray Gaussian, and so are the powers: the pixel's Toeplitz
// matrix of a dense, thin surface is ill-conditioned, and the float rounding
// of the phase and damping (about 3e-7) moved a pixel of a dense
// 500k-Gaussian 1080p scene by 6e-4 at three complex moments, against 5e-8
// with these in double.
template <int NH>
__device__ __forceinline__ void particle_trig_moments_d(const RayG& g, float tn, double* m) {
  constexpr double kSpanD = 5.654866776461628;  // 2 pi - theta
  const float mus = fmaxf(g.mu, tn);
  const float gp = warp_abs_d(mus, tn);
  const double musd = (double)mus;
  const double xq = 1.0 + 0.8 * musd;
  const double r = (1.0 + 0.8 * (double)tn) / xq;
  const double r15 = r * sqrt(r);
  const double gpd = 1.2 * r15 / xq;                                  // g_hat'(mu*)
  const double ggd = (1.0 - r15) + gpd * ((double)g.mu - musd);      // G, linearised at mu*
  const float a = (tn - g.mu) * kInvSqrt2 * fast_rcp(g.sig);
  const double ec = (double)erfc_fast(a);
  const double eb = (double)(g.sig * kTrigSpan * gp * kInvSqrt2 * 1.1283791670955126f * __expf(-a * a));
  const double amp = (double)(g.omega * g.sig * kSqrtHalfPi);
  double sn, cs;
  sincos(kSpanD * ggd, &sn, &cs);
  const double sa = (double)g.sig * kSpanD * gpd;
  const double d1 = exp(-0.5 * sa * sa);
  m[0] = amp * ec;
  double zr = 1.0, zi = 0.0, dk = 1.0, dstep = d1;
#pragma unroll
  for (int k = 1; k <= NH; ++k) {
    const double nr = zr * cs - zi * sn;
    zi = zr * sn + zi * cs;
    zr = nr;
    dk *= dstep;  // D^(k^2) = D^((k-1)^2) D^(2k-1)
    dstep *= d1 * d1;
    const double orr = ec, oi = (double)k * eb;
    const double f = amp * dk;
    m[2 * k - 1] = f * (zr * orr - zi * oi);
    m[2 * k] = f * (zr * oi + zi * orr);
  }
}

// Degenerate measures take the power moments' rule (hankel_factor) with the
// uniform measure in place of the normal, at a relative pivot of 1e-4 for two
// complex moments and 1e-3 for three: the circle has no affine freedom to
// condition the Toeplitz matrix, and depth measures on it are narrow arcs, so
// the float reconstruction needs the matrix well conditioned (with three
// moments at 1e-4, the float rounding of a moment moved F by up to 0.09).
template <int NH>
constexpr double pivot_rel_trig() {
  return NH == 2 ? 1e-4 : 1e-3;
}

// Cholesky of the Toeplitz matrix of c (c_0 = 1; c given as re/im), every
// relative pivot above pivot_rel_trig, and the factor when so.
template <int M>
__device__ __forceinline__ bool toeplitz_chol(const double* cr, const double* ci, double (&lr)[M][M],
                                              double (&li)[M][M]) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    double s = cr[0];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= lr[j][k] * lr[j][k] + li[j][k] * li[j][k];
    ok = ok && (s > pivot_rel_trig<M - 1>() * cr[0]);
    const double d = sqrt(fmax(s, 1e-300));
    lr[j][j] = d;
    li[j][j] = 0.0;
#pragma unroll
    for (int i = j + 1; i < M; ++i) {
      // T_ij = c_{j-i} = conj(c_{i-j}) for i > j
      double tr = cr[i - j], ti = -ci[i - j];
#pragma unroll
      for (int k = 0; k < j; ++k) {  // - L_ik conj(L_jk)
        tr -= lr[i][k] * lr[j][k] + li[i][k] * li[j][k];
        ti -= li[i][k] * lr[j][k] - lr[i][k] * li[j][k];
      }
      lr[i][j] = tr / d;
      li[i][j] = ti / d;
    }
  }
  return ok;
}

// Per-pixel set-up from the moment sums acc[0..2NH] (c_0, Re c_1, Im c_1, ..):
// returns the mixture weight with the uniform measure (0: none; -1: the
// identity factor, for moments without positive mass or non-finite ones).
template <int NH>
__device__ __forceinline__ double trig_factor(const double* acc, TrigLInv<NH>& out) {
  constexpr int M = NH + 1;
  double cr[M], ci[M];
  cr[0] = 1.0;
  ci[0] = 0.0;
  bool finite = acc[0] > 0.0 && isfinite(acc[0]);
#pragma unroll
  for (int k = 1; k <= NH; ++k) {
    cr[k] = acc[2 * k - 1] / acc[0];
    ci[k] = acc[2 * k] / acc[0];
    finite = finite && isfinite(cr[k]) && isfinite(ci[k]);
  }
  double lr[M][M], li[M][M];
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = 0; j < M; ++j) lr[i][j] = li[i][j] = 0.0;
  double eps = -1.0;
  if (finite) {
    if (toeplitz_chol<M>(cr, ci, lr, li)) {
      eps = 0.0;
    } else {
#pragma unroll 1
      for (int l = 0; l < kMixLevels && eps < 0.0; ++l) {
        double mr[M], mi[M];
        mr[0] = 1.0;
        mi[0] = 0.0;
#pragma unroll
        for (int k = 1; k < M; ++k) {
          mr[k] = (1.0 - kMixEps[l]) * cr[k];
          mi[k] = (1.0 - kMixEps[l]) * ci[k];
        }
        if (toeplitz_chol<M>(mr, mi, lr, li)) eps = kMixEps[l];
      }
    }
  }
  if (eps < 0.0) {
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
      for (int j = 0; j < M; ++j) {
        lr[i][j] = i == j ? 1.0 : 0.0;
        li[i][j] = 0.0;
      }
  }
  // inverse of the complex lower-triangular factor (real diagonal)
  double ir[M][M], ii[M][M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
#pragma unroll
    for (int j = 0; j < M; ++j) ir[i][j] = ii[i][j] = 0.0;
    const double inv = 1.0 / lr[i][i];
    ir[i][i] = inv;
#pragma unroll
    for (int j = 0; j < i; ++j) {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int k = j; k < i; ++k) {  // sum_k L_ik Linv_kj
        sr += lr[i][k] * ir[k][j] - li[i][k] * ii[k][j];
        si += lr[i][k] * ii[k][j] + li[i][k] * ir[k][j];
      }
      ir[i][j] = -sr * inv;
      ii[i][j] = -si * inv;
    }
  }
  int o = 0;
#pragma unroll
  for (int i = 0; i < M; ++i) {
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      out.re[o + j] = (float)ir[i][j];
      out.im[o + j] = (float)ii[i][j];
    }
    o += i + 1;
  }
  return eps;
}

// u = L^-1 conj(v(z)), v(z) = (1, z, .., z^NH)
template <int NH>
__device__ __forceinline__ void trig_linv_apply(const TrigLInv<NH>& L, cfl z, cfl* u) {
  cfl p[NH + 1];
  p[0] = {1.f, 0.f};
  const cfl zc = cconj(z);
#pragma unroll
  for (int k = 1; k <= NH; ++k) p[k] = cmul(p[k - 1], zc);
  int o = 0;
#pragma unroll
  for (int i = 0; i <= NH; ++i) {
    cfl s = {0.f, 0.f};
#pragma unroll
    for (int j = 0; j <= i; ++j) s = cadd(s, cmul({L.re[o + j], L.im[o + j]}, p[j]));
    u[i] = s;
    o += i + 1;
  }
}

template <int NH>
__device__ __forceinline__ float trig_christoffel(const TrigLInv<NH>& L, cfl z) {
  cfl u[NH + 1];
  trig_linv_apply<NH>(L, z, u);
  float s = 0.f;
#pragma unroll
  for (int i = 0; i <= NH; ++i) s += cabs2(u[i]);
  return fast_rcp(s);
}

// Order along the circle cut at angle 1.9 pi (the middle of the wrapping
// zone): z comes before w when its angle after the cut, in [0, 2 pi), is
// smaller. Both are turned by the cut; the half [0, pi) precedes [pi, 2 pi),
// and inside one half (angles less than pi apart) the sign of the cross
// product orders them.
struct CutPoint {
  float x, y;
  bool lower;  // angle after the cut in [pi, 2 pi)
};
__device__ __forceinline__ CutPoint cut_point(cfl z) {
  const float cr = 0.9510565162951535f, ci = 0.3090169943749474f;  // e^{-i cut}, cut = 1.9 pi
  CutPoint c;
  c.x = z.re * cr - z.im * ci;
  c.y = z.re * ci + z.im * cr;
  c.lower = c.y < 0.f || (c.y == 0.f && c.x < 0.f);
  return c;
}
__device__ __forceinline__ bool cut_before(const CutPoint& z, const CutPoint& w) {
  return z.lower != w.lower ? w.lower : (z.x * w.y - z.y * w.x > 0.f);
}

// Zeros of the cubic a_0 + a_1 z + a_2 z^2 + a_3 z^3 (complex coefficients):
// Laguerre's iteration from `start` (the query point w, on the circle and
// never a zero, or a zero of the previous edge's cubic, which lies near one
// of this cubic's) finds one zero (cubic convergence from almost any
// start), the quadratic left after dividing it out is solved in stable
// form, and every zero gets one Newton step on the cubic (the Laguerre zero
// leaves its loop converged, and one step takes a deflated zero from the
// rounding of the division to that of the cubic). The Laguerre
// step is taken as
//   3 p / (p' +- sqrt(2 (2 p'^2 - 3 p p''))),
// its usual form multiplied through by p, so that nothing divides by p: at a
// converged zero the fused evaluation of p can fall far below its rounding
// level, and the usual form's p' / p and its square then overflow float (a
// NaN zero). (Durand-Kerner from three fixed points of the circle failed to
// converge in ten steps on 0.2% of the queries of a 2,000-Gaussian 128x128
// image, where zeros cluster.)
__device__ __forceinline__ void cubic_roots(const cfl* a, cfl start, cfl* z) {
  const cfl ia = cdiv({1.f, 0.f}, a[3]);
  const cfl b0 = cmul(a[0], ia), b1 = cmul(a[1], ia), b2 = cmul(a[2], ia);
  auto p = [&](cfl x) __attribute__((always_inline)) {  // monic cubic
    return cadd(cmul(cadd(cmul(cadd(x, b2), x), b1), x), b0);
  };
  auto dp = [&](cfl x) __attribute__((always_inline)) {
    return cadd(cmul(cadd(cfl{3.f * x.re, 3.f * x.im}, cfl{2.f * b2.re, 2.f * b2.im}), x), b1);
  };
  cfl r = start;
#pragma unroll 1
  for (int it = 0; it < 8; ++it) {
    const cfl pz = p(r), d1 = dp(r);
    const cfl d2 = {6.f * r.re + 2.f * b2.re, 6.f * r.im + 2.f * b2.im};
    const cfl d11 = cmul(d1, d1), pd2 = cmul(pz, d2);
    const cfl sq = csqrt({4.f * d11.re - 6.f * pd2.re, 4.f * d11.im - 6.f * pd2.im});
    const cfl dpl = cadd(d1, sq), dmi = csub(d1, sq);
    const cfl den = cabs2(dpl) >= cabs2(dmi) ? dpl : dmi;
    if (!(cabs2(den) > 1e-30f)) break;  // a double zero at r (or a non-finite iterate)
    const cfl step = cdiv({3.f * pz.re, 3.f * pz.im}, den);
    r = csub(r, step);
    // close enough for the Newton polish below (|r| is about 1); a bound at
    // float resolution let iterates that stall at the rounding level run all
    // eight steps (and their wave with them) for no gain in the polished zeros
    if (cabs2(step) < 1e-10f) break;
  }
  // p(x) = (x - r)(x^2 + c1 x + c0)
  const cfl c1 = cadd(b2, r);
  const cfl c0 = cadd(b1, cmul(r, c1));
  const cfl disc = csub(cmul(c1, c1), cfl{4.f * c0.re, 4.f * c0.im});
  cfl sq = csqrt(disc);
  if (c1.re * sq.re + c1.im * sq.im < 0.f) sq = {-sq.re, -sq.im};
  const cfl q = {-0.5f * (c1.re + sq.re), -0.5f * (c1.im + sq.im)};
  z[0] = r;
  z[1] = q;
  z[2] = cabs2(q) > 1e-30f ? cdiv(c0, q) : cfl{0.f, 0.f};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const cfl d = dp(z[i]);
    if (cabs2(d) > 1e-30f) z[i] = csub(z[i], cdiv(p(z[i]), d));
  }
}

// The canonical representation through w = e^{i psi}: the NH other atoms,
// their flags (before w along the cut circle) and the weight lambda_0 at w;
// returns F = sum_{atoms before w} lambda_i + beta lambda_0. The weights sum
// to c_0 = 1, so with c of the NH atoms before w the sum is 0 (c = 0),
// 1 - lambda_0 (c = NH), the weight of the one atom before w (c = 1), or
// 1 - lambda_0 less the weight of the one atom after it (c = 2 of three):
// one Christoffel weight at most.
template <int NH>
struct TrigCanon {
  cfl z[NH];
  bool b[NH];
  float lam0;
};
// start (optional, in and out): the Laguerre start for three moments, the
// zero it found on return (the zeros move continuously along a Gaussian's
// edges, so the next edge starts close to one).
template <int NH>
__device__ __forceinline__ float trig_canon(const TrigLInv<NH>& L, float psi, float beta, TrigCanon<NH>& out,
                                            cfl* start = nullptr) {
  static_assert(NH == 2 || NH == 3, "the reconstruction is built for two or three complex moments");
  cfl w;
  sincosf(psi, &w.im, &w.re);
  cfl u[NH + 1];
  trig_linv_apply<NH>(L, w, u);
  float s0 = 0.f;
#pragma unroll
  for (int i = 0; i <= NH; ++i) s0 += cabs2(u[i]);
  const float lam0 = fast_rcp(s0);
  // a = L^-H u: a_j = sum_{i >= j} conj(Linv_ij) u_i
  cfl a[NH + 1];
#pragma unroll
  for (int j = 0; j <= NH; ++j) a[j] = {0.f, 0.f};
  int o = 0;
#pragma unroll
  for (int i = 0; i <= NH; ++i) {
#pragma unroll
    for (int j = 0; j <= i; ++j) a[j] = cadd(a[j], cmul(cconj({L.re[o + j], L.im[o + j]}), u[i]));
    o += i + 1;
  }
  if constexpr (NH == 2) {
    // zeros of a_0 + a_1 z + a_2 z^2 (stable form)
    const cfl disc = csub(cmul(a[1], a[1]), cmul({4.f * a[2].re, 4.f * a[2].im}, a[0]));
    cfl sq = csqrt(disc);
    if (a[1].re * sq.re + a[1].im * sq.im < 0.f) sq = {-sq.re, -sq.im};
    const cfl qq = {-0.5f * (a[1].re + sq.re), -0.5f * (a[1].im + sq.im)};
    out.z[0] = cdiv(qq, a[2]);
    out.z[1] = cdiv(a[0], qq);
  } else {
    const bool warm = start != nullptr && isfinite(start->re) && isfinite(start->im);
    cubic_roots(a, warm ? *start : w, out.z);
    if (start) *start = out.z[0];
  }
  const CutPoint cw = cut_point(w);
  out.lam0 = lam0;
  int cnt = 0;
#pragma unroll
  for (int i = 0; i < NH; ++i) {
    out.b[i] = cut_before(cut_point(out.z[i]), cw);
    cnt += out.b[i] ? 1 : 0;
  }
  // the one atom whose weight is needed: the atom before w (c = 1) or the
  // atom after it (c = NH - 1 = 2)
  const bool want = cnt == 1;
  cfl zs = out.z[NH - 1];
#pragma unroll
  for (int i = NH - 2; i >= 0; --i) zs = out.b[i] == want ? out.z[i] : zs;
  float ws = trig_christoffel<NH>(L, zs);
  ws = isfinite(ws) ? ws : 0.f;
  const float below = cnt == 0 ? 0.f : (cnt == NH ? 1.f - lam0 : (cnt == 1 ? ws : 1.f - lam0 - ws));
  return below + beta * lam0;
}

// F = sum_{atoms before w} lambda_i + beta lambda_0 at the query angle psi
template <int NH>
__device__ __forceinline__ float trig_F(const TrigLInv<NH>& L, float psi, float beta, cfl* start = nullptr) {
  TrigCanon<NH> c;
  return trig_canon<NH>(L, psi, beta, c, start);
}

// Adjoint of F through the moment equations sum_i lambda_i e^{i k theta_i} =
// c_k, k = 0..n (2n + 1 real equations; theta_0 = psi fixed; unknowns the
// n + 1 weights and the n other angles): the real trigonometric polynomial
//   Lambda(theta) = g_0 + sum_{k=1..n} (g_{2k-1} cos k theta + g_{2k} sin k theta)
// with Lambda(theta_i) = [atom i before w], Lambda'(theta_i) = 0 (i = 1..n)
// and Lambda(psi) = beta gives dF/d(c_0, Re c_1, Im c_1, .., Re c_n, Im c_n)
// = g, and dF/dpsi = -lambda_0 Lambda'(psi) (differentiate sum_i lambda_i
// Lambda(theta_i) = sum_k g_k c_k). The system is solved in closed form on
// the unit circle: with z = e^{i theta}, Q(z) = z^n Lambda(theta) is the
// complex polynomial of degree 2n with Q(z_i) = f_i z_i^n and
// Q'(z_i) = n f_i z_i^(n-1) (f_i the flag; Lambda'(theta_i) = 0 is
// z Q'(z) = n Q(z) there) and Q(w) = beta w^n. As for the power moments,
// Q = A + C P with P(z) = prod_i (z - z_i)^2, C = (beta w^n - A(w)) / P(w),
// and A the Hermite interpolant of the atoms' data: 0 (no flag set), z^n (all
// set), or built on the lone atom s of the minority side, A = R_s (one flag
// set) or z^n - R_s (all but one), where R_s(z) = q(z)^2 (u + v (z - s))
// vanishes to second order at the other atoms (q(z) = prod_{j != s} (z - z_j))
// and matches z^n to first order at s: u = s^n / q(s)^2,
// v = s^(n-1) (n - 2 s q'(s) / q(s)) / q(s)^2. Lambda is real, so its
// coefficients are read off the upper half of Q:
// g_0 = Re Q_n, g_{2k-1} = 2 Re Q_{n+k}, g_{2k} = -2 Im Q_{n+k}.
// Coincident nodes (a singular system) pass no gradient.
template <int NH>
__device__ __forceinline__ void trig_adjoint(float psi, const TrigCanon<NH>& c, float beta, float* g,
                                             float& dF_dpsi) {
  static_assert(NH == 2 || NH == 3, "the adjoint is built for two or three complex moments");
  cfl w;
  sincosf(psi, &w.im, &w.re);
  cfl z[NH];
  int cnt = 0;
#pragma unroll
  for (int i = 0; i < NH; ++i) {
    const float nz = rsqrtf(fmaxf(cabs2(c.z[i]), 1e-30f));
    z[i] = {c.z[i].re * nz, c.z[i].im * nz};
    cnt += c.b[i] ? 1 : 0;
  }
  // A = s0 z^n + s1 R_s; the lone atom carries the flag `want`
  const float s1 = cnt == 1 ? 1.f : ((NH == 3 && cnt == 2) ? -1.f : 0.f);
  const float s0 = (cnt == NH || s1 < 0.f) ? 1.f : 0.f;
  const bool want = cnt == 1;
  const cfl w2 = cmul(w, w);
  const cfl wn = NH == 2 ? w2 : cmul(w2, w);
  cfl Qn, Qh[NH];  // Q_n and Q_{n+1}, .., Q_{2n}
  bool ok;
  if constexpr (NH == 2) {
    const bool l1 = c.b[1] == want && c.b[0] != want;  // lone atom z_1 (else z_0)
    const cfl s = l1 ? z[1] : z[0], a = l1 ? z[0] : z[1];
    // q(z) = z - a; u = s^2 / q(s)^2, v = -2 a s / q(s)^3
    const cfl qs = csub(s, a);
    const bool okq = s1 == 0.f || cabs2(qs) > 1e-20f;
    const cfl iq = okq && s1 != 0.f ? cdiv({1.f, 0.f}, qs) : cfl{0.f, 0.f};
    const cfl iq2 = cmul(iq, iq);
    const cfl u = cmul(cmul(s, s), iq2);
    const cfl v = cmul(cmul(cmul(a, s), {-2.f * iq2.re, -2.f * iq2.im}), iq);
    const cfl up = csub(u, cmul(v, s));  // R(z) = (z - a)^2 (up + v z)
    const cfl R2 = csub(up, cmul(cfl{2.f * a.re, 2.f * a.im}, v)), R3 = v;
    const cfl wa = csub(w, a);
    const cfl Rw = cmul(cmul(wa, wa), cadd(up, cmul(v, w)));
    // p(z) = (z - z_0)(z - z_1) = z^2 + p1 z + p0, P = p^2
    const cfl p1 = {-(z[0].re + z[1].re), -(z[0].im + z[1].im)}, p0 = cmul(z[0], z[1]);
    const cfl pw = cmul(csub(w, z[0]), csub(w, z[1]));
    const cfl Pw = cmul(pw, pw);
    ok = okq && cabs2(pw) > 1e-20f;
    const cfl Aw = {s0 * wn.re + s1 * Rw.re, s0 * wn.im + s1 * Rw.im};
    const cfl C = ok ? cdiv(csub({beta * wn.re, beta * wn.im}, Aw), Pw) : cfl{0.f, 0.f};
    const cfl P2 = cadd(cmul(p1, p1), {2.f * p0.re, 2.f * p0.im}), P3 = {2.f * p1.re, 2.f * p1.im};
    Qn = cadd({s0 + s1 * R2.re, s1 * R2.im}, cmul(C, P2));
    Qh[0] = cadd({s1 * R3.re, s1 * R3.im}, cmul(C, P3));
    Qh[1] = C;
  } else {
    const bool l1 = c.b[1] == want && c.b[0] != want && c.b[2] != want;
    const bool l2 = c.b[2] == want && c.b[0] != want && c.b[1] != want;
    // (s, a, b) = (z0, z1, z2), (z1, z0, z2) or (z2, z0, z1)
    const cfl s = l1 ? z[1] : (l2 ? z[2] : z[0]);
    const cfl a = (l1 || l2) ? z[0] : z[1];
    const cfl b = l2 ? z[1] : z[2];
    // q(z) = (z - a)(z - b) = z^2 + q1 z + q0
    const cfl q1 = {-(a.re + b.re), -(a.im + b.im)}, q0 = cmul(a, b);
    const cfl qs = cmul(csub(s, a), csub(s, b));
    const bool okq = s1 == 0.f || cabs2(qs) > 1e-20f;
    const cfl iq = okq && s1 != 0.f ? cdiv({1.f, 0.f}, qs) : cfl{0.f, 0.f};
    const cfl iq2 = cmul(iq, iq);
    const cfl ss = cmul(s, s);
    const cfl u = cmul(cmul(ss, s), iq2);
    // v = s^2 (3 q(s) - 2 s (2 s + q1)) / q(s)^3  (q'(s) = 2 s + q1)
    const cfl t = csub({3.f * qs.re, 3.f * qs.im}, cmul({2.f * s.re, 2.f * s.im}, cadd({2.f * s.re, 2.f * s.im}, q1)));
    const cfl v = cmul(cmul(ss, t), cmul(iq2, iq));
    const cfl up = csub(u, cmul(v, s));  // R(z) = q(z)^2 (up + v z)
    // q^2 = z^4 + 2 q1 z^3 + (q1^2 + 2 q0) z^2 + ..
    const cfl q2c2 = cadd(cmul(q1, q1), {2.f * q0.re, 2.f * q0.im}), q2c3 = {2.f * q1.re, 2.f * q1.im};
    const cfl R3 = cadd(cmul(up, q2c3), cmul(v, q2c2));
    const cfl R4 = cadd(up, cmul(v, q2c3));
    const cfl R5 = v;
    const cfl qw = cmul(csub(w, a), csub(w, b));
    const cfl Rw = cmul(cmul(qw, qw), cadd(up, cmul(v, w)));
    // p(z) = (z - z_0)(z - z_1)(z - z_2) = z^3 + p2 z^2 + p1 z + p0, P = p^2
    const cfl p2 = {-(z[0].re + z[1].re + z[2].re), -(z[0].im + z[1].im + z[2].im)};
    const cfl z01 = cmul(z[0], z[1]);
    const cfl p1 = cadd(z01, cmul(cadd(z[0], z[1]), z[2]));
    const cfl p0 = {-cmul(z01, z[2]).re, -cmul(z01, z[2]).im};
    const cfl pw = cmul(cmul(csub(w, z[0]), csub(w, z[1])), csub(w, z[2]));
    const cfl Pw = cmul(pw, pw);
    ok = okq && cabs2(pw) > 1e-20f;
    const cfl Aw = {s0 * wn.re + s1 * Rw.re, s0 * wn.im + s1 * Rw.im};
    const cfl C = ok ? cdiv(csub({beta * wn.re, beta * wn.im}, Aw), Pw) : cfl{0.f, 0.f};
    const cfl P3 = {2.f * (p0.re + (p1.re * p2.re - p1.im * p2.im)), 2.f * (p0.im + (p1.re * p2.im + p1.im * p2.re))};
    const cfl P4 = cadd(cmul(p2, p2), {2.f * p1.re, 2.f * p1.im}), P5 = {2.f * p2.re, 2.f * p2.im};
    Qn = cadd({s0 + s1 * R3.re, s1 * R3.im}, cmul(C, P3));
    Qh[0] = cadd({s1 * R4.re, s1 * R4.im}, cmul(C, P4));
    Qh[1] = cadd({s1 * R5.re, s1 * R5.im}, cmul(C, P5));
    Qh[2] = C;
  }
  g[0] = ok ? Qn.re : 0.f;
#pragma unroll
  for (int k = 1; k <= NH; ++k) {
    g[2 * k - 1] = ok ? 2.f * Qh[k - 1].re : 0.f;
    g[2 * k] = ok ? -2.f * Qh[k - 1].im : 0.f;
  }
  float dl = 0.f;
  cfl wk = w;
#pragma unroll
  for (int k = 1; k <= NH; ++k) {
    dl += (float)k * (-g[2 * k - 1] * wk.im + g[2 * k] * wk.re);
    wk = cmul(wk, w);
  }
  dF_dpsi = -c.lam0 * dl;
}

// sum_k dm[k] d c_k / d(mu, Sigma, omega) for one Gaussian's moments (as
// particle_trig_moments_d computes them; dm over (c_0, Re c_1, Im c_1, ..)),
// from the derivatives of their factors: amplitude omega Sigma sqrt(pi / 2),
// erfc(a), the first-order erf term k b e^{-a^2}, the damping D^(k^2) and the
// phase e^{i k alpha_1 G}.
template <int NH>
__device__ __forceinline__ void trig_moment_grads(const RayG& g, float tn, const float* dm, float* out) {
  const bool unc = g.mu > tn;
  const float mus = fmaxf(g.mu, tn);
  const float gp = warp_abs_d(mus, tn);
  const float gpp = unc ? -2.f * gp * fast_rcp(1.f + 0.8f * mus) : 0.f;  // g_hat'' (0 when linearised at t_n)
  const float G = warp_abs(mus, tn) + gp * (g.mu - mus);
  const float is = fast_rcp(g.sig);
  const float a = (tn - g.mu) * kInvSqrt2 * is;
  const float E = __expf(-a * a);
  const float ec = erfc_fast(a);
  const float amp1 = g.sig * kSqrtHalfPi;  // amplitude over omega
  const float amp = g.omega * amp1;
  const float Cb = kTrigSpan * kInvSqrt2 * 1.1283791670955126f;
  const float eb = Cb * g.sig * gp * E;
  const float sa = g.sig * kTrigSpan * gp;
  // d/dmu (index 0) and d/dSigma (index 1) of the factors
  const float da[2] = {-kInvSqrt2 * is, -a * is};
  const float dgp[2] = {gpp, 0.f};
  const float dphi[2] = {kTrigSpan * gp, 0.f};
  const float damp_rel[2] = {0.f, is};
  const float dsa[2] = {g.sig * kTrigSpan * gpp, kTrigSpan * gp};
  float dec[2], deb[2];
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    const float dE = -2.f * a * E * da[d];
    dec[d] = -1.1283791670955126f * E * da[d];
    deb[d] = Cb * ((d == 1 ? gp * E : 0.f) + g.sig * (dgp[d] * E + gp * dE));
  }
  float gd[2];
#pragma unroll
  for (int d = 0; d < 2; ++d) gd[d] = dm[0] * amp * (dec[d] + ec * damp_rel[d]);
  float gom = dm[0] * amp1 * ec;
  float sn, cs;
  sincosf(kTrigSpan * G, &sn, &cs);
  cfl zk = {1.f, 0.f};
#pragma unroll
  for (int k = 1; k <= NH; ++k) {
    zk = cmul(zk, {cs, sn});
    const float kf = (float)k;
    const float Dk = __expf(-0.5f * kf * kf * sa * sa);
    const cfl base = cmul(zk, {ec * Dk, kf * eb * Dk});  // c_k / amp
    gom += amp1 * (dm[2 * k - 1] * base.re + dm[2 * k] * base.im);
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const float dlnD = -kf * kf * sa * dsa[d];
      const cfl t1 = cmul(base, {damp_rel[d] + dlnD, kf * dphi[d]});
      const cfl t2 = cmul(zk, {dec[d] * Dk, kf * deb[d] * Dk});
      gd[d] += amp * (dm[2 * k - 1] * (t1.re + t2.re) + dm[2 * k] * (t1.im + t2.im));
    }
  }
  out[0] = gd[0];
  out[1] = gd[1];
  out[2] = gom;
}

// Quadrature of Eq. 7 for one Gaussian against the circle's reconstruction:
// the edge at depth t queries the angle (2 pi - theta) g_hat(t); the optical
// depth is a running maximum along the edges.
template <int NH, int NQ>
__device__ __forceinline__ float particle_quadrature_trig(const RayG& g, const TrigLInv<NH>& L, float m0, float tn,
                                                          const RenderArgs& a, QEdges<NQ>& e) {
  cfl start = {__builtin_nanf(""), 0.f};  // the first edge starts from its query point
#pragma unroll
  for (int j = 0; j < NQ; ++j) {
    e.off[j] = a.kappa * g.sig * a.xq[j];
    float t = g.mu + e.off[j];
    e.cl[j] = t < tn;
    t = e.cl[j] ? tn : t;
    e.y[j] = kTrigSpan * warp_abs(t, tn);
    const float r = (t - g.mu) * fast_rcp(g.sig);
    e.sj[j] = g.omega * (e.cl[j] ? exp_neg_half(r * r) : a.eq[j]);
    const float tj = m0 * trig_F<NH>(L, e.y[j], a.beta, &start);
    e.tau[j] = (j == 0 || tj > e.tau[j > 0 ? j - 1 : 0]) ? tj : e.tau[j > 0 ? j - 1 : 0];
  }
  return quad_sum<NQ>(g, tn, e);
}

}  // namespace mb
