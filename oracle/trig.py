"""Trigonometric moments of the ray density and bounds on the circle (float64).

TEST INFRASTRUCTURE: see the package docstring.

Sec. 3.2 (Eqs. 13-14) and App. C: the warped depth is placed on the unit
circle at the angle phi(t) = (2 pi - theta) g_hat(t), and the density moments
are the Fourier coefficients

    m~_k = sum_j int_{t_n}^{inf} e^{i k phi(t)} sigma_j(t) dt,   k = 0..n.

Per particle, with g_hat linearised at the mean and t_f -> infinity (Eq. 14),

    (m~_k)_j ~ omega sqrt(pi/2) Sigma e^{i alpha G - Sigma^2 beta^2 / 2} (1 - erf(v_n)),
    alpha = k (2 pi - theta),  beta = alpha G',
    v_n = (t_n - mu) / (sqrt2 Sigma) - i Sigma beta / sqrt2,

and erf of the complex argument a - i b is taken to first order in b
(App. C): erf(a - i b) ~ erf(a) - i b (2 / sqrt(pi)) e^{-a^2}. m~_0 is the
exact optical depth.

The paper leaves the reconstruction from these moments to the cited works.
Readings taken here (each listed in the design notes):

* theta, the wrapping zone: THETA = 0.2 pi (the physical depths [t_n, inf)
  fill the arc [0, 1.8 pi), the arc (1.8 pi, 2 pi) stays empty).
* The warp is linearised at max(mu, t_n), as for the power moments.
* "K moments" are n = K / 2 complex moments m~_1..m~_n beside m~_0: the same
  2n + 1 real numbers a K-moment power basis stores.
* Reconstruction: the canonical representation through the query point
  w = e^{i psi} on the circle, i.e. the Gauss-Szego quadrature of the
  Toeplitz matrix T_jk = c_{k-j} of the normalised moments c = m~ / m~_0:
  atoms at w and at the n zeros of the kernel polynomial
  q(z) = v(z)^T T^-1 conj(v(w)), v(z) = (1, z, .., z^n) (all on the unit
  circle), with the Christoffel weights 1 / (v(z)^T T^-1 conj(v(z))). As in
  the cited line of work on trigonometric moments, the atoms are ordered
  along the circle cut in the middle of the wrapping zone (angle
  2 pi - theta / 2): L sums the weights of the atoms before the query, U adds
  the query's own weight (the largest mass any measure with these moments
  can hold at w), and tau = m~_0 ((1 - beta) L + beta U). Unlike the power
  moments' L and U these are estimates, not bounds: the circle has no end,
  and atoms in the wrapping zone are counted on one side of the cut.
  Along a Gaussian's quadrature edges the optical depth is made
  non-decreasing (running maximum, a later edge taking over only when
  strictly larger), as for the learned surrogate, because the estimates
  need not grow with depth.
* A Toeplitz matrix singular to working precision (a nearly atomic measure)
  is mixed with the uniform measure on the circle, c' = (1 - eps) c +
  eps (1, 0, .., 0), for the first eps of bounds.MIX_EPS whose matrix has
  every relative Cholesky pivot above pivot_rel_trig(n) (the rule of
  bounds.degenerate_mixture; the uniform measure is the rotation-invariant
  stand-in for the normal). The threshold is 1e-4 for two complex moments
  and 1e-3 for three, not the power moments' 1e-5: the circle has no affine
  freedom to condition the matrix, and depth measures on it are narrow arcs,
  so a float32 reconstruction needs the Toeplitz matrix conditioned well
  (with three moments at 1e-4, a relative moment change of 3e-7, the float
  rounding of a moment, moved F by up to 0.09; at 1e-3 by 3e-5).

The ordering at the cut is a discrete decision: an atom on one side of the
cut counts before every query, on the other side after every query, so the
optical depth jumps by m~_0 times its weight as it crosses. cut_margin gives
the distance of the nearest atom to the cut; a result whose queries have an
atom closer than CUT_BAND is decided by the rounding of its inputs (a float
rounding of the ray Gaussians, about 3e-7 relative, moved the atoms within
0.01 rad of the cut by at most 1.5e-4 rad over 1,500 pixels of a
500k-Gaussian 1080p scene).
"""
from __future__ import annotations

import math

import numpy as np
import torch
from scipy import special

from .bounds import MIX_EPS
from .geometry import DT
from .moments import warp, warp_prime

THETA = 0.2 * math.pi
PIVOT_REL_TRIG = {2: 1e-4, 3: 1e-3}
CUT_BAND = 2e-4  # radians


def pivot_rel_trig(n: int) -> float:
    """Relative Cholesky pivot below which n + 1 complex moments count as
    degenerate (see the module docstring)."""
    return PIVOT_REL_TRIG[n]


CT = torch.complex128


def angle_of(t, t_near: float, theta: float = THETA):
    """phi(t) = (2 pi - theta) g_hat(t): depth on the circle."""
    return (2.0 * math.pi - theta) * warp(t, t_near)


def particle_trig_moments(mu, sigma, omega, t_near: float, n: int, theta: float = THETA,
                          exact_erf: bool = False):
    """Eq. 14 for k = 0..n: complex [..., n+1]. ``exact_erf`` evaluates the
    complex erf exactly (scipy's Faddeeva-based erf; no autograd) instead of
    the first-order expansion, for the pins."""
    mu_star = torch.clamp_min(mu, t_near)
    gp = warp_prime(mu_star, t_near)
    g = warp(mu_star, t_near) + gp * (mu - mu_star)
    a = (t_near - mu) / (math.sqrt(2.0) * sigma)
    amp = omega * sigma * math.sqrt(math.pi / 2.0)
    out = [torch.complex(amp * torch.special.erfc(a), torch.zeros_like(a))]
    for k in range(1, n + 1):
        alpha = k * (2.0 * math.pi - theta)
        beta = alpha * gp
        b = sigma * beta / math.sqrt(2.0)
        damp = torch.exp(-0.5 * sigma * sigma * beta * beta)
        if exact_erf:
            v = a.detach().numpy() - 1j * b.detach().numpy()
            one_minus = torch.as_tensor(1.0 - special.erf(v), dtype=CT)
        else:
            one_minus = torch.complex(torch.special.erfc(a),
                                      b * (2.0 / math.sqrt(math.pi)) * torch.exp(-a * a))
        phase = torch.complex(torch.cos(alpha * g), torch.sin(alpha * g))
        out.append(amp * damp * phase * one_minus)
    return torch.stack(out, dim=-1)


def toeplitz(c: torch.Tensor, n: int) -> torch.Tensor:
    """T_jk = c_{k-j} (c_{-m} = conj(c_m)), j, k = 0..n."""
    rows = []
    for j in range(n + 1):
        rows.append(torch.stack([c[..., k - j] if k >= j else torch.conj(c[..., j - k])
                                 for k in range(n + 1)], dim=-1))
    return torch.stack(rows, dim=-2)


def _powers(z: torch.Tensor, n: int) -> torch.Tensor:
    return torch.stack([z ** k for k in range(n + 1)], dim=-1)


def _pivots_pass(c: np.ndarray, n: int) -> np.ndarray:
    """Every Cholesky pivot of T (rows of normalised c, c_0 = 1) above
    pivot_rel_trig(n) times its diagonal entry."""
    idx = np.arange(n + 1)
    d = idx[None, :] - idx[:, None]  # k - j
    t = np.where(d >= 0, c[..., np.abs(d)], np.conj(c[..., np.abs(d)]))
    ok = np.ones(c.shape[:-1], bool)
    lc = np.zeros(t.shape, complex)
    for j in range(n + 1):
        piv = (t[..., j, j] - (np.abs(lc[..., j, :j]) ** 2).sum(-1)).real
        ok &= piv > pivot_rel_trig(n) * t[..., j, j].real
        dj = np.sqrt(np.maximum(piv, 1e-300))
        lc[..., j, j] = dj
        for i in range(j + 1, n + 1):
            lc[..., i, j] = (t[..., i, j] - (lc[..., i, :j] * np.conj(lc[..., j, :j])).sum(-1)) / dj
    return ok


def uniform_mixture(c: torch.Tensor, n: int):
    """The normalised moments the reconstruction uses (c, or its mixture with
    the uniform measure) and the mixture weight per row (0: none)."""
    with torch.no_grad():
        cn = c.detach().numpy()
        level = np.where(_pivots_pass(cn, n), 0.0, -1.0)
        unif = np.zeros_like(cn)
        unif[..., 0] = 1.0
        for e in MIX_EPS:
            todo = level < 0
            if not todo.any():
                break
            level = np.where(todo & _pivots_pass((1 - e) * cn + e * unif, n), e, level)
        eps = torch.as_tensor(level, dtype=DT)
    e = eps.clamp_min(0.0)[..., None].to(CT)
    unif_t = torch.zeros_like(c)
    unif_t[..., 0] = 1.0
    return torch.where(eps[..., None] > 0, (1 - e) * c + e * unif_t, c), eps


def _circle_roots(coef: torch.Tensor) -> torch.Tensor:
    """Roots of sum_k coef[..., k] z^k (complex, degree n >= 1), from the
    companion eigenvalues, polished by Newton steps, with one more Newton step
    at the held root to carry dz/dcoef = -(dq/dcoef)(z) / q'(z) to autograd."""
    n = coef.shape[-1] - 1
    c = coef.detach().numpy()
    if n == 1:
        z0 = (-c[..., 0] / c[..., 1])[..., None]
    else:
        monic = c[..., :n] / c[..., n:n + 1]
        comp = np.zeros(c.shape[:-1] + (n, n), complex)
        comp[..., 1:, :-1] = np.eye(n - 1)
        comp[..., :, -1] = -monic
        z0 = np.linalg.eigvals(comp)
    z = torch.as_tensor(z0, dtype=CT)
    cd = coef.detach()

    def q_dq(zv, cc):
        q = torch.zeros_like(zv)
        dq = torch.zeros_like(zv)
        for k in range(n, -1, -1):
            dq = dq * zv + q
            q = q * zv + cc[..., k:k + 1]
        return q, dq

    for _ in range(3):
        q, dq = q_dq(z, cd)
        z = z - torch.where(dq != 0, q / dq, torch.zeros_like(q))
    q, dq = q_dq(z, coef)
    return z - q / dq.detach()


def circle_canonical(c: torch.Tensor, w: torch.Tensor, n: int):
    """Atoms z [Q, n+1] (z[:, 0] = w) and Christoffel weights lam [Q, n+1]
    of the canonical representation through w (|w| = 1) of the normalised
    moments c [Q, n+1] (c_0 = 1)."""
    t = toeplitz(c, n)
    vw = _powers(w, n)
    a = torch.linalg.solve(t, torch.conj(vw).unsqueeze(-1)).squeeze(-1)  # q(z) = v(z)^T a
    roots = _circle_roots(a)
    z = torch.cat([w.unsqueeze(-1), roots], dim=-1)
    vz = _powers(z, n)                                                  # [Q, n+1 atoms, n+1]
    tinv_vz = torch.linalg.solve(t.unsqueeze(-3), torch.conj(vz).unsqueeze(-1)).squeeze(-1)
    lam = 1.0 / (vz * tinv_vz).sum(-1).real
    return z, lam


def arc_position(z: torch.Tensor, theta: float = THETA) -> torch.Tensor:
    """Position of e^{i phi} along the circle cut in the middle of the
    wrapping zone: (phi - (2 pi - theta / 2)) mod 2 pi, in [0, 2 pi)."""
    phi = torch.atan2(z.imag, z.real)
    return torch.remainder(phi - (2.0 * math.pi - 0.5 * theta), 2.0 * math.pi)


def trig_bound_tau(m: torch.Tensor, psi: torch.Tensor, n: int, beta: float, theta: float = THETA):
    """Optical depth at the query angle psi from the trigonometric moments
    m [Q, n+1] (complex, m_0 real): tau = m_0 ((1 - beta) L + beta U) with the
    reconstruction described above; 0 where m_0 = 0. Returns (tau, L, U)."""
    m0 = m[..., 0].real
    pos = m0 > 0
    safe = torch.where(pos, m0, torch.ones_like(m0)).to(CT)
    unit = torch.zeros_like(m)
    unit[..., 0] = 1.0
    c = torch.where(pos[..., None], m / safe[..., None], unit)
    c, _ = uniform_mixture(c, n)
    w = torch.complex(torch.cos(psi), torch.sin(psi))
    z, lam = circle_canonical(c, w, n)
    s = arc_position(z, theta)
    below = (s[..., 1:] < s[..., :1]).to(DT)
    lower = (lam[..., 1:] * below).sum(-1)
    upper = lower + lam[..., 0]
    tau = m0 * ((1.0 - beta) * lower + beta * upper)
    return torch.where(pos, tau, torch.zeros_like(tau)), lower, upper


def cut_margin(m: torch.Tensor, psi: torch.Tensor, n: int, theta: float = THETA) -> torch.Tensor:
    """Distance (radians) from the cut to the nearest atom other than the
    query of the canonical representation that trig_bound_tau uses at each
    query psi; infinite where m_0 = 0."""
    with torch.no_grad():
        m0 = m[..., 0].real
        pos = m0 > 0
        safe = torch.where(pos, m0, torch.ones_like(m0)).to(CT)
        unit = torch.zeros_like(m)
        unit[..., 0] = 1.0
        c = torch.where(pos[..., None], m / safe[..., None], unit)
        c, _ = uniform_mixture(c, n)
        w = torch.complex(torch.cos(psi), torch.sin(psi))
        z, _ = circle_canonical(c, w, n)
        s = arc_position(z[..., 1:], theta)
        d = torch.minimum(s, 2.0 * math.pi - s).amin(-1)
        return torch.where(pos, d, torch.full_like(d, math.inf))


def degenerate_flags(m: torch.Tensor, n: int) -> torch.Tensor:
    """Mixture weight of the degenerate-measure rule per row of complex
    moments m (0: none)."""
    c = m / m[..., :1].real.to(CT)
    _, eps = uniform_mixture(c, n)
    return eps
