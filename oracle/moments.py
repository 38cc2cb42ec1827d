"""Depth warp and warped power moments of the ray density (float64).

TEST INFRASTRUCTURE: see the package docstring.
"""
from __future__ import annotations

import math

import torch

LAMBDA = -1.5  # power-transform parameter, Sec. 3.2


def power_transform(x, lam: float = LAMBDA):
    """Barron's power transform f_lambda(x) = |lam-1|/lam ((x/|lam-1| + 1)^lam - 1)
    (the transform the paper cites for its warp; its slope at 0 is 1)."""
    a = abs(lam - 1.0)
    return (a / lam) * ((x / a + 1.0) ** lam - 1.0)


def _f_inf(lam: float = LAMBDA) -> float:
    """lim_{x->inf} f_lambda(x) for lam < 0 (the far bound t_f -> infinity)."""
    return -abs(lam - 1.0) / lam


def warp(t, t_near: float, lam: float = LAMBDA):
    """g_hat(t) = (f(t) - f(t_n)) / (f(t_f) - f(t_n)) with f(t) = f_lambda(2t),
    lambda = -1.5 and t_f -> infinity (Sec. 3.2); maps [t_n, inf) to [0, 1)."""
    fn = power_transform(2.0 * t_near, lam)
    return (power_transform(2.0 * t, lam) - fn) / (_f_inf(lam) - fn)


def warp_prime(t, t_near: float, lam: float = LAMBDA):
    """d g_hat / dt, using f_lambda'(x) = (x/|lam-1| + 1)^(lam-1)."""
    a = abs(lam - 1.0)
    fn = power_transform(2.0 * t_near, lam)
    return 2.0 * (2.0 * t / a + 1.0) ** (lam - 1.0) / (_f_inf(lam) - fn)


def linearised_warp(mu, t_near: float, centre, scale):
    """First-order Taylor expansion of the warp at the particle mean
    (App. C), expressed in the affine moment variable y = (g_hat - centre)/scale.

    Returns (G, G') so that y(t) ~ G + G' (t - mu). For a mean in front of the
    near bound the warp is expanded at max(mu, t_n) instead (reading: the
    warp is undefined for 1 + 0.8 mu <= 0), i.e. G = y(mu*) + y'(mu*)(mu - mu*).
    """
    mu_star = torch.clamp_min(mu, t_near)
    gp = warp_prime(mu_star, t_near) / scale
    g = (warp(mu_star, t_near) - centre) / scale + gp * (mu - mu_star)
    return g, gp


def particle_moments(mu, sigma, omega, t_near: float, n_moments: int,
                     centre, scale):
    """Warped power moments of one ray Gaussian, Eqs. 10-12 with t_f -> inf
    (App. C), in the moment variable y = (g_hat - centre) / scale:

        m_0 = omega Sigma sqrt(pi/2) (1 - erf(b_n))
        m_1 = G m_0 + G' omega Sigma^2 exp(-b_n^2)
        m_k = G m_{k-1} + (k-1) G'^2 Sigma^2 m_{k-2} + G' omega Sigma^2 u_n^(k-1) exp(-b_n^2)

    with b_n = (t_n - mu)/(sqrt2 Sigma), u_n = G + G'(t_n - mu).  The boundary
    term enters with a plus sign: the appendix's t_f -> infinity limit of the
    integration by parts gives +, the minus in the main-text Eq. 11 is read as a
    typo; Eq. 12's u_n (not v_n) is used.  An affine moment variable leaves the
    reconstructed bounds unchanged, so ``centre``/``scale`` only condition the
    arithmetic.  Returns [..., K+1]."""
    g, gp = linearised_warp(mu, t_near, centre, scale)
    bn = (t_near - mu) / (math.sqrt(2.0) * sigma)
    e = torch.exp(-bn * bn)
    s2 = sigma * sigma
    m = [omega * sigma * math.sqrt(math.pi / 2.0) * torch.special.erfc(bn)]
    bnd = gp * omega * s2 * e          # boundary term without u_n^(k-1)
    m.append(g * m[0] + bnd)
    un = g + gp * (t_near - mu)
    un_pow = un
    for k in range(2, n_moments + 1):
        m.append(g * m[k - 1] + (k - 1) * gp * gp * s2 * m[k - 2] + bnd * un_pow)
        un_pow = un_pow * un
    return torch.stack(m, dim=-1)
