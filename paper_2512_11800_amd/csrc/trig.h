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
// b = Sigma alpha_1 G' / sqrt 2, a = (t_n - mu) / (sqrt2 Sigma). The powers are
// taken in double from the float primitives, so that every pair's moment
// vector is, to double rounding, that of one Gaussian (the Toeplitz matrix of
// a narrow measure keeps its small pivots).
template <int NH>
__device__ __forceinline__ void particle_trig_moments_d(const RayG& g, float tn, double* m) {
  const float mus = fmaxf(g.mu, tn);
  const float gp = warp_abs_d(mus, tn);
  const float gg = warp_abs(mus, tn) + gp * (g.mu - mus);
  const float a = (tn - g.mu) * kInvSqrt2 * fast_rcp(g.sig);
  const double ec = (double)erfc_fast(a);
  const double eb = (double)(g.sig * kTrigSpan * gp * kInvSqrt2 * 1.1283791670955126f * __expf(-a * a));
  const double amp = (double)(g.omega * g.sig * kSqrtHalfPi);
  float sn, cs;
  sincosf(kTrigSpan * gg, &sn, &cs);
  const float sa = g.sig * kTrigSpan * gp;
  const double d1 = (double)__expf(-0.5f * sa * sa);
  m[0] = amp * ec;
  double zr = 1.0, zi = 0.0, dk = 1.0, dstep = d1;
#pragma unroll
  for (int k = 1; k <= NH; ++k) {
    const double nr = zr * (double)cs - zi * (double)sn;
    zi = zr * (double)sn + zi * (double)cs;
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
// uniform measure in place of the normal, at a relative pivot of 1e-4: the
// circle has no affine freedom to condition the Toeplitz matrix, and depth
// measures on it are narrow arcs, so the float reconstruction needs the
// matrix conditioned to about 1e5 or better.
constexpr double kPivotRelTrig = 1e-4;

// Cholesky of the Toeplitz matrix of c (c_0 = 1; c given as re/im), every
// relative pivot above kPivotRelTrig, and the factor when so.
template <int M>
__device__ __forceinline__ bool toeplitz_chol(const double* cr, const double* ci, double (&lr)[M][M],
                                              double (&li)[M][M]) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    double s = cr[0];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= lr[j][k] * lr[j][k] + li[j][k] * li[j][k];
    ok = ok && (s > kPivotRelTrig * cr[0]);
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

// position along the circle after the cut, in [0, 2 pi)
__device__ __forceinline__ float arc_pos(cfl z) {
  // rotate by -cut
  const float cr = 0.9510565162951535f, ci = 0.3090169943749474f;  // e^{-i cut}, cut = 1.9 pi
  const float xr = z.re * cr - z.im * ci, xi = z.re * ci + z.im * cr;
  const float a = atan2f(xi, xr);
  return a < 0.f ? a + 6.283185307179586f : a;
}

// The canonical representation through w = e^{i psi}: the other atoms, their
// flags (before w along the cut circle) and the weight lambda_0 at w; returns
// F = sum_{atoms before w} lambda_i + beta lambda_0.
struct TrigCanon {
  cfl z1, z2;
  bool b1, b2;
  float lam0;
};
template <int NH>
__device__ __forceinline__ float trig_canon(const TrigLInv<NH>& L, float psi, float beta, TrigCanon& out) {
  static_assert(NH == 2, "the trigonometric reconstruction is built for two complex moments");
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
  // zeros of a_0 + a_1 z + a_2 z^2 (stable form)
  const cfl disc = csub(cmul(a[1], a[1]), cmul({4.f * a[2].re, 4.f * a[2].im}, a[0]));
  cfl sq = csqrt(disc);
  if (a[1].re * sq.re + a[1].im * sq.im < 0.f) sq = {-sq.re, -sq.im};
  const cfl qq = {-0.5f * (a[1].re + sq.re), -0.5f * (a[1].im + sq.im)};
  const cfl z1 = cdiv(qq, a[2]), z2 = cdiv(a[0], qq);
  const float pw = arc_pos(w);
  out.z1 = z1;
  out.z2 = z2;
  out.b1 = arc_pos(z1) < pw;
  out.b2 = arc_pos(z2) < pw;
  out.lam0 = lam0;
  float f = beta * lam0;
  f += out.b1 ? trig_christoffel<NH>(L, z1) : 0.f;
  f += out.b2 ? trig_christoffel<NH>(L, z2) : 0.f;
  return f;
}

// F = sum_{atoms before w} lambda_i + beta lambda_0 at the query angle psi
template <int NH>
__device__ __forceinline__ float trig_F(const TrigLInv<NH>& L, float psi, float beta) {
  TrigCanon c;
  return trig_canon<NH>(L, psi, beta, c);
}

// Adjoint of F through the moment equations sum_i lambda_i e^{i k theta_i} =
// c_k, k = 0, 1, 2 (five real equations; theta_0 = psi fixed; unknowns the
// three weights and the two other angles): the real trigonometric polynomial
//   Lambda(theta) = g0 + g1 cos theta + g2 sin theta + g3 cos 2theta + g4 sin 2theta
// with Lambda(theta_i) = [atom i before w], Lambda'(theta_i) = 0 (i = 1, 2)
// and Lambda(psi) = beta gives dF/d(c_0, Re c_1, Im c_1, Re c_2, Im c_2) = g,
// and dF/dpsi = -lambda_0 Lambda'(psi) (differentiate sum_i lambda_i
// Lambda(theta_i) = sum_k g_k c_k). The 5 x 5 system is solved by Gaussian
// elimination with partial pivoting; a singular one (coincident atoms) passes
// no gradient.
__device__ __forceinline__ void trig_adjoint(float psi, const TrigCanon& c, float beta, float* g, float& dF_dpsi) {
  float sp, cp;
  sincosf(psi, &sp, &cp);
  const float n1 = rsqrtf(fmaxf(cabs2(c.z1), 1e-30f)), n2 = rsqrtf(fmaxf(cabs2(c.z2), 1e-30f));
  const float c1 = c.z1.re * n1, s1 = c.z1.im * n1, c2 = c.z2.re * n2, s2 = c.z2.im * n2;
  float M[5][6] = {
      {1.f, cp, sp, cp * cp - sp * sp, 2.f * cp * sp, beta},
      {1.f, c1, s1, c1 * c1 - s1 * s1, 2.f * c1 * s1, c.b1 ? 1.f : 0.f},
      {1.f, c2, s2, c2 * c2 - s2 * s2, 2.f * c2 * s2, c.b2 ? 1.f : 0.f},
      {0.f, -s1, c1, -4.f * c1 * s1, 2.f * (c1 * c1 - s1 * s1), 0.f},
      {0.f, -s2, c2, -4.f * c2 * s2, 2.f * (c2 * c2 - s2 * s2), 0.f}};
  bool ok = true;
#pragma unroll
  for (int col = 0; col < 5; ++col) {
    // partial pivoting over the rows below (selects keep it branch free)
#pragma unroll
    for (int r = col + 1; r < 5; ++r) {
      const bool sw = fabsf(M[r][col]) > fabsf(M[col][col]);
#pragma unroll
      for (int k = col; k < 6; ++k) {
        const float t = M[col][k];
        M[col][k] = sw ? M[r][k] : t;
        M[r][k] = sw ? t : M[r][k];
      }
    }
    ok = ok && fabsf(M[col][col]) > 1e-7f;
    const float ip = ok ? fast_rcp(M[col][col]) : 0.f;
#pragma unroll
    for (int r = col + 1; r < 5; ++r) {
      const float f = M[r][col] * ip;
#pragma unroll
      for (int k = col + 1; k < 6; ++k) M[r][k] = fmaf(-f, M[col][k], M[r][k]);
    }
  }
#pragma unroll
  for (int r = 4; r >= 0; --r) {
    float v = M[r][5];
#pragma unroll
    for (int k = r + 1; k < 5; ++k) v = fmaf(-M[r][k], g[k], v);
    g[r] = ok ? v * fast_rcp(M[r][r]) : 0.f;
  }
  const float dl = -g[1] * sp + g[2] * cp - 4.f * g[3] * cp * sp + 2.f * g[4] * (cp * cp - sp * sp);
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
#pragma unroll
  for (int j = 0; j < NQ; ++j) {
    e.off[j] = a.kappa * g.sig * a.xq[j];
    float t = g.mu + e.off[j];
    e.cl[j] = t < tn;
    t = e.cl[j] ? tn : t;
    e.y[j] = kTrigSpan * warp_abs(t, tn);
    const float r = (t - g.mu) * fast_rcp(g.sig);
    e.sj[j] = g.omega * (e.cl[j] ? exp_neg_half(r * r) : a.eq[j]);
    const float tj = m0 * trig_F<NH>(L, e.y[j], a.beta);
    e.tau[j] = (j == 0 || tj > e.tau[j > 0 ? j - 1 : 0]) ? tj : e.tau[j > 0 ? j - 1 : 0];
  }
  return quad_sum<NQ>(g, tn, e);
}

}  // namespace mb
