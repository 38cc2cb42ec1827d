"""Moment-bound reconstruction of the optical depth (float64).

TEST INFRASTRUCTURE: see the package docstring.

Sec. 3.2: given the moments b_0..b_2n of a measure, the canonical
representation through the query eta is the (n+1)-atom measure with one atom
at x_0 = eta and the same moments. Its other atoms x_1..x_n are the roots of
the kernel polynomial K(x) = v(x)^T H^-1 v(eta) (H the Hankel matrix of the
moments, v(x) = (1, x, .., x^n)), its weights solve the Vandermonde system of
the moment equations, and
    L(eta) = sum_{x_i < eta} w_i,   U(eta) = sum_{x_i <= eta} w_i.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .geometry import DT


def hankel(b: torch.Tensor, n: int) -> torch.Tensor:
    """H_ij = b_{i+j}, i, j = 0..n, batched over the leading dimension."""
    idx = torch.arange(n + 1)
    return b[..., idx[:, None] + idx[None, :]]


def powers(x: torch.Tensor, n: int) -> torch.Tensor:
    return torch.stack([x ** k for k in range(n + 1)], dim=-1)


def _poly_roots(coef: torch.Tensor) -> torch.Tensor:
    """Real roots of sum_k coef[..., k] x^k (all real for a positive definite
    Hankel matrix), differentiable in ``coef``.

    The roots come from the eigenvalues of the companion matrix (numpy),
    are polished by Newton steps, and then one more Newton step is taken
    with the root held constant, which carries the exact first derivative
    dx/dc = -(dp/dc)(x) / p'(x) to autograd."""
    n = coef.shape[-1] - 1
    c = coef.detach().cpu().numpy()
    monic = c[..., :n] / c[..., n:n + 1]
    comp = np.zeros(c.shape[:-1] + (n, n))
    comp[..., 1:, :-1] = np.eye(n - 1)
    comp[..., :, -1] = -monic
    x0 = np.sort(np.real(np.linalg.eigvals(comp)), axis=-1)
    x = torch.as_tensor(x0, dtype=DT)
    cd = coef.detach()

    def p_and_dp(xv, cc):
        p = torch.zeros_like(xv)
        dp = torch.zeros_like(xv)
        for k in range(n, -1, -1):
            dp = dp * xv + p
            p = p * xv + cc[..., k:k + 1]
        return p, dp

    for _ in range(3):
        p, dp = p_and_dp(x, cd)
        step = torch.where(dp != 0, p / dp, torch.zeros_like(p))
        x = x - step
    p, dp = p_and_dp(x, coef)
    return x - p / dp.detach()


def canonical_representation(b: torch.Tensor, eta: torch.Tensor, n: int):
    """Atoms and weights of the canonical representation through ``eta``.

    ``b``: [Q, 2n+1] moments (b_0 = total mass); ``eta``: [Q].
    Returns (x [Q, n+1] with x[:,0] = eta, w [Q, n+1])."""
    h = hankel(b, n)
    v_eta = powers(eta, n)
    c = torch.linalg.solve(h, v_eta.unsqueeze(-1)).squeeze(-1)
    roots = _poly_roots(c)
    x = torch.cat([eta.unsqueeze(-1), roots], dim=-1)
    vand = powers(x, n).transpose(-1, -2)          # [Q, k, i] = x_i^k
    w = torch.linalg.solve(vand, b[..., :n + 1].unsqueeze(-1)).squeeze(-1)
    return x, w


# Degenerate measures (a reading: the paper assumes a positive definite
# Hankel matrix). A sum of Gaussians has positive definite Hankel matrices in
# exact arithmetic, but a nearly atomic one (ray Gaussians far thinner than
# their separation) is singular to working precision. The measure counts as
# degenerate when a Cholesky pivot of the Hankel matrix of its standardised
# moments E[((y - mean) / sd)^k] (independent of the affine moment variable)
# is at most PIVOT_REL times its diagonal entry (1e-5: well above the float32
# rounding a GPU's per-pair moments carry into these pivots, about 1e-7, so a
# float32 implementation can decide it reliably); it is then replaced by the
# mixture (1 - eps) mu + eps N(mean, sd^2) with the normal distribution of its
# own mean and variance, for the first eps in MIX_EPS whose mixture passes the
# same test. The mixture is a valid measure, transforms with the moment
# variable, and is differentiable in the moments.
PIVOT_REL = 1e-5
MIX_EPS = (1e-3, 1e-2, 1e-1, 1.0)


def normal_moments(mean: torch.Tensor, var: torch.Tensor, k_max: int):
    """[..., k_max + 1] moments E[(mean + sd Z)^k] of N(mean, var):
    n_k = mean n_{k-1} + (k - 1) var n_{k-2}."""
    out = [torch.ones_like(mean), mean]
    for k in range(2, k_max + 1):
        out.append(mean * out[k - 1] + (k - 1) * var * out[k - 2])
    return torch.stack(out[:k_max + 1], dim=-1)


def standardised_moments(b: torch.Tensor) -> torch.Tensor:
    """E[((y - mean) / sd)^k] from the moments b_k = E[y^k] (b_0 = 1), by the
    binomial expansion of (y - mean)^k."""
    k_max = b.shape[-1] - 1
    mean = b[..., 1]
    sd = torch.sqrt(b[..., 2] - mean * mean)
    out = []
    for k in range(k_max + 1):
        c = sum(math.comb(k, j) * b[..., j] * (-mean) ** (k - j) for j in range(k + 1))
        out.append(c / sd ** k)
    return torch.stack(out, dim=-1)


def _pivots_pass(c: np.ndarray, n: int) -> np.ndarray:
    """Whether every Cholesky pivot of the Hankel matrix of c (rows) exceeds
    PIVOT_REL times its diagonal entry."""
    h = c[..., np.arange(n + 1)[:, None] + np.arange(n + 1)[None, :]]
    ok = np.ones(c.shape[:-1], bool)
    lc = np.zeros(h.shape)
    for j in range(n + 1):
        piv = h[..., j, j] - (lc[..., j, :j] ** 2).sum(-1)
        ok &= piv > PIVOT_REL * h[..., j, j]
        d = np.sqrt(np.maximum(piv, 1e-300))
        lc[..., j, j] = d
        for i in range(j + 1, n + 1):
            lc[..., i, j] = (h[..., i, j] - (lc[..., i, :j] * lc[..., j, :j]).sum(-1)) / d
    return ok


def degenerate_mixture(b: torch.Tensor, n: int):
    """The moments the bounds use (b itself, or the mixture above) and the
    mixture weight per row (0: none; -1: no positive variance or non-finite
    moments, where no bound is defined)."""
    with torch.no_grad():
        bd = b.detach()
        var = bd[..., 2] - bd[..., 1] ** 2
        fin = torch.isfinite(bd).all(-1) & (var > 0)
        eps = torch.full(bd.shape[:-1], -1.0, dtype=DT)
        if bool(fin.any()):
            c = standardised_moments(torch.where(fin[..., None], bd, _unit_measure_moments(bd.shape, n)))
            cn = c.numpy()
            sn = _unit_measure_moments(bd.shape, n).numpy()
            level = np.where(_pivots_pass(cn, n), 0.0, -1.0)
            for e in MIX_EPS:
                todo = level < 0
                if not todo.any():
                    break
                passed = _pivots_pass((1 - e) * cn + e * sn, n)
                level = np.where(todo & passed, e, level)
            eps = torch.where(fin, torch.as_tensor(level, dtype=DT), eps)
    mean = b[..., 1]
    nm = normal_moments(mean, b[..., 2] - mean * mean, b.shape[-1] - 1)
    e = eps.clamp_min(0.0)[..., None]
    return torch.where(eps[..., None] > 0, (1 - e) * b + e * nm, b), eps


def bound_tau(m: torch.Tensor, eta: torch.Tensor, n: int, beta: float):
    """Optical depth at ``eta`` from the moments m_0..m_2n of the ray density:
    tau = (1 - beta) L + beta U (Sec. 3.2; the printed "T(tau) = ..." is read
    as the interpolated optical depth, since L and U bound the cumulative
    density), with L, U the bounds of the measure with moments m.  Computed
    on the normalised moments b = m / m_0 and scaled back by m_0; tau = 0 where
    m_0 = 0.  Returns (tau, L, U) with L, U normalised."""
    m0 = m[..., 0]
    pos = m0 > 0
    b = torch.where(pos[..., None], m / torch.where(pos, m0, torch.ones_like(m0))[..., None],
                    _unit_measure_moments(m.shape, n))
    b, _ = degenerate_mixture(b, n)
    x, w = canonical_representation(b, eta, n)
    below = (x[..., 1:] < eta[..., None]).to(DT)
    lower = (w[..., 1:] * below).sum(-1)
    upper = lower + w[..., 0]
    tau = m0 * ((1.0 - beta) * lower + beta * upper)
    return torch.where(pos, tau, torch.zeros_like(tau)), lower, upper


def _unit_measure_moments(shape, n):
    """Moments of a standard normal, used as a harmless stand-in where a
    pixel has no density (its result is replaced by 0)."""
    k = shape[-1]
    mom = [1.0, 0.0]
    for j in range(2, k):
        mom.append((j - 1) * mom[j - 2])
    return torch.tensor(mom, dtype=DT).expand(shape)
