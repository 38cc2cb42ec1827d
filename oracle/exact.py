"""Ground truth for image quality: the volume rendering equation evaluated
without the moment approximation.

TEST INFRASTRUCTURE: see the package docstring.

Along a pixel ray every Gaussian is the 1D Gaussian of Eqs. 4-6, so the
optical depth has the closed form (Eq. 10's zeroth moment, cut at t)

    tau(t) = sum_j w_j Sigma_j sqrt(pi/2) [erf((t - mu_j) / (sqrt2 Sigma_j))
                                          - erf((t_n - mu_j) / (sqrt2 Sigma_j))],

and the radiance of Eq. 2 with the emission of Eq. 3 is

    L = sum_i (L_e)_i int_{t_n}^{inf} sigma_i(t) e^{-tau(t)} dt + e^{-tau(inf)} L_bg.

The integral is taken by composite Gauss-Legendre quadrature on intervals cut
at every Gaussian's mu_j + k Sigma_j for a ladder of k, so each interval is
short against the finest structure that overlaps it. Every Gaussian whose
total optical depth beyond t_n exceeds ``min_depth`` takes part (not only the
proxy-covered ones: this is the reference the method approximates).
"""
from __future__ import annotations

import math

import numpy as np
import torch
from scipy.special import erf

from .geometry import DT, camera_matrices, pixel_directions, quat_to_rot, ray_gaussian, sh_rgb
from .render import scene_tensors

_LADDER = np.array([-8, -6, -4, -3, -2, -1.5, -1, -0.5, 0, 0.5, 1, 1.5, 2, 3, 4, 6, 8], np.float64)
_SQ = math.sqrt(math.pi / 2)


def optical_depth(t, mu, sigma, omega, t_near: float):
    """tau(t) for depths t [T] and ray Gaussians (mu, sigma, omega) [G]: [T]."""
    t = np.asarray(t, np.float64)[:, None]
    a = erf((t - mu[None, :]) / (math.sqrt(2) * sigma[None, :]))
    a0 = erf((t_near - mu) / (math.sqrt(2) * sigma))
    return ((a - a0[None, :]) * (omega * sigma * _SQ)[None, :]).sum(1)


def exact_ray(mu, sigma, omega, rgb, t_near: float, background, nodes: int = 8, chunk: int = 16384):
    """Radiance [3] of Eq. 2 along one ray with ray Gaussians mu, sigma, omega
    [G] and colours rgb [G, 3]."""
    mu, sigma, omega = (np.asarray(v, np.float64) for v in (mu, sigma, omega))
    rgb = np.asarray(rgb, np.float64)
    bg = np.asarray(background, np.float64)
    if mu.size == 0:
        return bg.copy()
    tot = omega * sigma * _SQ * (1.0 - erf((t_near - mu) / (math.sqrt(2) * sigma)))
    t_inf = math.exp(-tot.sum())
    cuts = (mu[:, None] + sigma[:, None] * _LADDER[None, :]).reshape(-1)
    cuts = np.unique(np.concatenate([[t_near], cuts[cuts > t_near]]))
    if cuts.size < 2:
        return t_inf * bg
    xg, wg = np.polynomial.legendre.leggauss(nodes)
    lo, hi = cuts[:-1], cuts[1:]
    half = 0.5 * (hi - lo)
    t = ((lo + hi)[:, None] * 0.5 + half[:, None] * xg[None, :]).reshape(-1)
    w = (half[:, None] * wg[None, :]).reshape(-1)
    out = np.zeros(3)
    for s in range(0, t.size, chunk):
        ts = t[s:s + chunk]
        tau = optical_depth(ts, mu, sigma, omega, t_near)
        dens = omega[None, :] * np.exp(-0.5 * ((ts[:, None] - mu[None, :]) / sigma[None, :]) ** 2)
        out += ((w[s:s + chunk] * np.exp(-tau))[:, None] * (dens @ rgb)).sum(0)
    return out + t_inf * bg


def exact_pixels(scene, cam, pixels, min_depth: float = 1e-10, nodes: int = 8):
    """Ground-truth radiance [P, 3] of the listed pixels (flat y * W + x)."""
    scene_t = scene_tensors(scene)
    _, _, origin = camera_matrices(cam)
    rgb_all = sh_rgb(scene_t["colors"], scene.sh_degree, scene_t["means"], origin).detach().numpy()
    rot = quat_to_rot(scene_t["quats"])
    pix = np.asarray(pixels, np.int64)
    out = np.zeros((pix.size, 3))
    with torch.no_grad():
        for i, p in enumerate(pix):
            px = torch.tensor([int(p % cam.width)])
            py = torch.tensor([int(p // cam.width)])
            d = pixel_directions(cam, px, py).expand(scene.n, 3)
            mu, sigma, omega = ray_gaussian(origin, d, scene_t["means"], rot, scene_t["scales"],
                                            scene_t["densities"])
            mu, sigma, omega = mu.numpy(), sigma.numpy(), omega.numpy()
            tot = omega * sigma * _SQ * (1.0 - erf((cam.t_near - mu) / (math.sqrt(2) * sigma)))
            keep = tot > min_depth
            out[i] = exact_ray(mu[keep], sigma[keep], omega[keep], rgb_all[keep], cam.t_near,
                               cam.background, nodes)
    return out


def psnr(a, b, peak: float = 1.0) -> float:
    """10 log10(peak^2 / mean squared difference)."""
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10.0 * math.log10(peak * peak / mse)
