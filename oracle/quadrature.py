"""Per-Gaussian radiance quadrature and opacity rescaling (float64).

TEST INFRASTRUCTURE: see the package docstring.
"""
from __future__ import annotations

import numpy as np
import torch
from scipy.stats import norm

from .geometry import DT


def normal_quantiles(n_intervals: int) -> torch.Tensor:
    """Standard-normal samples x_j = Phi^-1(u_j) for the N+1 interval edges
    (App. B, sample spacing). The paper applies Phi^-1 to uniformly spaced
    samples of [0, 1]; the endpoints would map to +-infinity, so the reading
    taken is the midpoints u_j = (j - 1/2)/(N+1), j = 1..N+1."""
    u = (np.arange(1, n_intervals + 2) - 0.5) / (n_intervals + 1)
    return torch.as_tensor(norm.ppf(u), dtype=DT)


def _phi(x: torch.Tensor) -> torch.Tensor:
    """(1 - exp(-x)) / x, continued by 1 at x = 0."""
    small = x.abs() < 1e-6
    xs = torch.where(small, torch.ones_like(x), x)
    exact = -torch.expm1(-xs) / xs
    series = 1.0 - x / 2.0 + x * x / 6.0
    return torch.where(small, series, exact)


def particle_quadrature(mu, sigma, omega, tau_at, t_near: float, kappa: float,
                        n_intervals: int, warp_y):
    """Eq. 7 for one particle (App. B):

        L_i ~ sum_{j=1..N} (T(t_j) - T(t_{j+1})) sigma_i(t_j) / sigma(t_j) (L_e)_i,
        sigma(t_j) = (tau(t_{j+1}) - tau(t_j)) / Delta_j,

    with edges t_j = mu + kappa Sigma x_j clamped to [t_n, inf) and
    sigma_i(t_j) = omega exp(-(t_j - mu)^2 / (2 Sigma^2)) at the left edge of
    each interval.  Since T(t_{j+1}) = T(t_j) exp(-Delta tau_j), each term equals
    T_j Delta_j phi(Delta tau_j) sigma_i(t_j) with phi(x) = (1 - e^-x)/x, the
    form used here (it is defined where Delta tau_j = 0).

    ``tau_at(y)`` evaluates the reconstructed optical depth at moment
    variable y (shape [P, N+1]); ``warp_y(t)`` maps depth to y.
    Returns (q [P], tau [P, N+1], t [P, N+1]); q multiplies (r, g, b, 1)."""
    x = normal_quantiles(n_intervals)
    t = torch.clamp_min(mu[:, None] + kappa * sigma[:, None] * x[None, :], t_near)
    tau = tau_at(warp_y(t))
    trans = torch.exp(-tau)
    dt = t[:, 1:] - t[:, :-1]
    dtau = tau[:, 1:] - tau[:, :-1]
    sig_i = omega[:, None] * torch.exp(-(t[:, :-1] - mu[:, None]) ** 2
                                       / (2.0 * sigma[:, None] ** 2))
    q = (trans[:, :-1] * dt * _phi(dtau) * sig_i).sum(-1)
    return q, tau, t


def rescale(m0, s_rgb, o, eps: float, background):
    """Eq. 15: L = (1 - e^-m0) / max(eps, O) * sum_i L_i + e^-m0 L_bg."""
    bg = torch.as_tensor(background, dtype=DT)
    alpha = -torch.expm1(-m0)
    return alpha[:, None] * s_rgb / torch.clamp_min(o, eps)[:, None] \
        + torch.exp(-m0)[:, None] * bg


def interval_depth(mu, sigma, omega, t):
    """Optical depth of each particle alone over its quadrature intervals
    [t_j, t_{j+1}] (App. E, regularisation): the integral of
    omega exp(-(s - mu)^2 / (2 Sigma^2)) over the interval, in closed form
    omega Sigma sqrt(pi/2) (erf(b_{j+1}) - erf(b_j)), b = (t - mu) / (sqrt2 Sigma).
    t: [P, N+1] edges; returns [P, N]."""
    b = (t - mu[:, None]) / (np.sqrt(2.0) * sigma[:, None])
    e = torch.special.erf(b)
    return (omega * sigma * np.sqrt(np.pi / 2.0))[:, None] * (e[:, 1:] - e[:, :-1])


def consistency_penalty(mu, sigma, omega, tau, t):
    """P_i = sum_j max(0, tau_ij - (tau(t_{j+1}) - tau(t_j)))^2 over the
    quadrature intervals (App. E, regularisation; Sec. 3.4): the reconstructed
    optical depth gained over an interval may not fall below that of any one
    particle alone. tau, t: [P, N+1] at the edges; returns [P]."""
    tij = interval_depth(mu, sigma, omega, t)
    r = torch.clamp_min(tij - (tau[:, 1:] - tau[:, :-1]), 0.0)
    return (r * r).sum(-1)
