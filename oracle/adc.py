"""Adaptive density control of the density-based medium (Sec. 4.2's training
paragraph, App. E "Adaptive Density Control"), float64.

TEST INFRASTRUCTURE: see the package docstring.

* ``view_independent_opacity`` -- a particle's opacity seen along its
  shortest axis through its centre, the pruning criterion.
* ``density_from_opacity`` -- its inverse with the mean scale, used to
  initialise peak densities.
* ``split_objective`` -- the 1D opacity-contribution mismatch whose minimiser
  gives the split parameters; ``SPLIT_GAMMA`` and ``SPLIT_DELTA`` are the
  values the appendix prints (a pin checks that they sit at its minimum).
* ``plan`` / ``apply`` -- one densification step: prune by opacity, then
  clone (both copies at half density) or split (two particles along the
  longest axis) by the accumulated absolute mean gradient and the size.
"""
from __future__ import annotations

import math

import numpy as np

from .geometry import quat_to_rot

SPLIT_GAMMA = 0.6385502815246582
SPLIT_DELTA = 0.6128153090966912

PRUNE, KEEP, CLONE, SPLIT = 0, 1, 2, 3


def view_independent_opacity(scales, densities):
    """o = 1 - exp(-sqrt(2 pi) w min(s)): the optical depth of the particle
    along its shortest axis through its centre is w s_min sqrt(2 pi) (the
    exponent of Eq. 5 vanishes there, and the two erf terms of the
    single-particle optical depth are bounded by 2)."""
    s = np.asarray(scales, np.float64)
    w = np.asarray(densities, np.float64)
    return 1.0 - np.exp(-math.sqrt(2.0 * math.pi) * w * s.min(axis=-1))


def density_from_opacity(opacity, scales):
    """Peak density from an initial opacity, solving the expression above with
    the mean scale in place of the smallest (the appendix's initialisation)."""
    o = np.asarray(opacity, np.float64)
    s = np.asarray(scales, np.float64)
    return -np.log1p(-o) / (math.sqrt(2.0 * math.pi) * s.mean(axis=-1))


def opacity_contribution(sig, t):
    """T(-inf -> t) sigma(t) of a 1D density sampled on the uniform grid t
    (trapezoidal cumulative optical depth)."""
    dt = t[1] - t[0]
    tau = np.concatenate([[0.0], np.cumsum(0.5 * (sig[1:] + sig[:-1]) * dt)])
    return np.exp(-tau) * sig


def split_objective(c, gamma, half_width=12.0, n=24001):
    """Integral of (T_old sigma_old - T_new sigma_new)^2 over the standardised
    axis, sigma_old = exp(-t^2/2) and sigma_new the two particles of scale
    gamma at +-c (1 - gamma) (the appendix's constrained form, where the
    shrunken particles' confidence intervals stay inside the original's)."""
    t = np.linspace(-half_width, half_width, n)
    d = c * (1.0 - gamma)
    old = np.exp(-0.5 * t * t)
    new = np.exp(-(t - d) ** 2 / (2 * gamma * gamma)) + np.exp(-(t + d) ** 2 / (2 * gamma * gamma))
    r = opacity_contribution(old, t) - opacity_contribution(new, t)
    return float(np.sum(r * r) * (t[1] - t[0]))


def plan(scales, densities, grad_acc, grad_count, min_opacity, grad_threshold, split_scale):
    """Action per particle: PRUNE if its view-independent opacity is below
    min_opacity; otherwise CLONE or SPLIT when the norm of its accumulated
    absolute mean gradient per counted view exceeds grad_threshold (SPLIT if
    its largest scale exceeds split_scale), else KEEP. Returns (action,
    output offsets, output count)."""
    s = np.asarray(scales, np.float64)
    o = view_independent_opacity(s, densities)
    cnt = np.asarray(grad_count, np.float64)
    g = np.linalg.norm(np.asarray(grad_acc, np.float64), axis=-1) / np.maximum(cnt, 1.0)
    dens = (cnt > 0) & (g > grad_threshold)
    big = s.max(axis=-1) > split_scale
    action = np.where(o < min_opacity, PRUNE, np.where(dens, np.where(big, SPLIT, CLONE), KEEP))
    outs = np.array([0, 1, 2, 2])[action]
    offsets = np.concatenate([[0], np.cumsum(outs)[:-1]]).astype(np.int64)
    return action.astype(np.int32), offsets, int(outs.sum())


def apply(means, scales, quats, densities, colors, action):
    """The particle set after one step, in input order: a kept particle once;
    a cloned one twice at half its peak density (the two copies together are
    the original density); a split one as two particles at
    mean -+ SPLIT_DELTA s_max e_max with that scale shrunk by SPLIT_GAMMA
    (e_max the axis of the largest scale), everything else copied."""
    import torch
    means = np.asarray(means, np.float64)
    scales = np.asarray(scales, np.float64)
    quats = np.asarray(quats, np.float64)
    dens = np.asarray(densities, np.float64)
    cols = np.asarray(colors, np.float64)
    rot = quat_to_rot(torch.as_tensor(quats)).numpy()
    out = {k: [] for k in ("means", "scales", "quats", "densities", "colors")}

    def emit(m, s, q, w, c):
        out["means"].append(m)
        out["scales"].append(s)
        out["quats"].append(q)
        out["densities"].append(w)
        out["colors"].append(c)

    for i, a in enumerate(np.asarray(action)):
        if a == KEEP:
            emit(means[i], scales[i], quats[i], dens[i], cols[i])
        elif a == CLONE:
            emit(means[i], scales[i], quats[i], 0.5 * dens[i], cols[i])
            emit(means[i], scales[i], quats[i], 0.5 * dens[i], cols[i])
        elif a == SPLIT:
            k = int(np.argmax(scales[i]))
            axis = rot[i][:, k]
            off = SPLIT_DELTA * scales[i][k] * axis
            s_new = scales[i].copy()
            s_new[k] *= SPLIT_GAMMA
            emit(means[i] - off, s_new, quats[i], dens[i], cols[i])
            emit(means[i] + off, s_new, quats[i], dens[i], cols[i])
    return {k: np.array(v) for k, v in out.items()}
