"""Forward pass over a set of pixels, and its gradient by float64 autograd.

TEST INFRASTRUCTURE: see the package docstring.

Per pixel (Sec. 3, App. B/D): the Gaussians whose proxy rectangle covers the
pixel centre contribute their warped moments (Eqs. 10-12) to the pixel's
moment vector; each of them is then integrated with the quadrature of Eq. 7
against the optical depth reconstructed from those moments, and the sums of
(r, g, b, 1)-weighted contributions are rescaled by Eq. 15.  Everything is
additive over Gaussians, so the result does not depend on their order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, Optional

import numpy as np
import torch

from .bounds import bound_tau, degenerate_mixture
from .geometry import DT, camera_matrices, pixel_directions, quat_to_rot, ray_gaussian, sh_rgb
from .moments import particle_moments, warp
from .proxy import MARGIN_TOL, ORIENT_EPS, covering_pairs, screen_proxy
from .quadrature import consistency_penalty, particle_quadrature, rescale
from .trig import CUT_BAND, angle_of, cut_margin, degenerate_flags, particle_trig_moments, trig_bound_tau

PARAMS = ("means", "scales", "quats", "densities", "colors")


def scene_tensors(scene, requires_grad: bool = False) -> Dict[str, torch.Tensor]:
    """float64 leaf tensors of the scene parameters."""
    out = {}
    for k in PARAMS:
        t = torch.as_tensor(np.asarray(getattr(scene, k)), dtype=DT).clone()
        t.requires_grad_(requires_grad)
        out[k] = t
    return out


@dataclass
class PixelResult:
    image: torch.Tensor      # [P,3]
    s_rgb: torch.Tensor      # [P,3]  sum_i q_i rgb_i
    opacity: torch.Tensor    # [P]    O = sum_i q_i
    moments: torch.Tensor    # [P,K+1] in the pixel's moment variable
    centre: torch.Tensor     # [P] warp value at the pixel's moment origin
    scale: torch.Tensor      # [P] warp scale of the pixel's moment variable
    ambiguous: torch.Tensor  # [P] bool (parity protocol)
    n_pairs: int
    pair_slot: torch.Tensor
    pair_gid: torch.Tensor
    pair_q: torch.Tensor
    pair_y: torch.Tensor     # [pairs, N+1] moment variable at the quadrature edges
    pair_tau: torch.Tensor   # [pairs, N+1] reconstructed optical depth there
    penalty: torch.Tensor    # [P] consistency penalty sum_i P_i (App. E)
    fallback: torch.Tensor   # [P] bool: the pixel's measure is degenerate (bounds.degenerate_mixture)


def _standardised_basis(slot, mu, sigma, omega, t_near, n_pix):
    """The affine moment variable y = (g_hat - centre) / scale with centre and
    scale the mean and standard deviation of the pixel's (linearised) warped
    density.  The bounds do not depend on this choice (an increasing affine
    change of variable maps canonical representations onto each other); it
    only keeps the Hankel matrix well conditioned."""
    with torch.no_grad():
        raw = particle_moments(mu, sigma, omega, t_near, 2, 0.0, 1.0)
        acc = torch.zeros(n_pix, 3, dtype=DT).index_add_(0, slot, raw)
        m0 = acc[:, 0]
        ok = m0 > 0
        m0s = torch.where(ok, m0, torch.ones_like(m0))
        mean = acc[:, 1] / m0s
        var = (acc[:, 2] / m0s - mean * mean).clamp_min(0.0)
        scale = torch.sqrt(var)
        scale = torch.where(ok & (scale > 0), scale, torch.ones_like(scale))
        mean = torch.where(ok, mean, torch.zeros_like(mean))
    return mean, scale


def render_pixels(scene_t, scene, cam, opts, px: torch.Tensor, py: torch.Tensor,
                  proxy=None, margin_tol: float = MARGIN_TOL, orient_eps: float = ORIENT_EPS,
                  tau_model=None) -> PixelResult:
    """Render the listed pixels (all pairs of each listed pixel are formed, so
    every listed pixel is complete). ``tau_model(mom_q, y)`` replaces the
    reconstruction of Sec. 3.2 when given (optical depth at queries y [Q] of
    pixels with moments mom_q [Q, K+1]), e.g. by a learned surrogate."""
    n_pix = px.shape[0]
    k_mom = opts.n_moments
    n_half = k_mom // 2
    t_near = cam.t_near
    if proxy is None:
        proxy = screen_proxy(scene_t, cam, opts.conf_c)
    slot, gid, amb = covering_pairs(proxy, cam, px, py, margin_tol=margin_tol,
                                    full_coverage=opts.full_coverage, orient_eps=orient_eps)
    _, _, origin = camera_matrices(cam)

    means = scene_t["means"]
    rgb_all = sh_rgb(scene_t["colors"], scene.sh_degree, means, origin)
    d = pixel_directions(cam, px[slot], py[slot])
    rot = quat_to_rot(scene_t["quats"][gid])
    mu, sigma, omega = ray_gaussian(origin, d, means[gid], rot, scene_t["scales"][gid],
                                    scene_t["densities"][gid])

    n_edge = opts.n_intervals + 1
    if getattr(opts, "basis", "power") == "trigonometric":
        return _render_pixels_trig(scene_t, cam, opts, n_pix, slot, gid, amb, mu, sigma, omega,
                                   rgb_all, tau_model)
    centre, scale = _standardised_basis(slot, mu, sigma, omega, t_near, n_pix)
    mom_pair = particle_moments(mu, sigma, omega, t_near, k_mom, centre[slot], scale[slot])
    mom = torch.zeros(n_pix, k_mom + 1, dtype=DT).index_add(0, slot, mom_pair)

    mom_q = mom[slot].repeat_interleave(n_edge, dim=0)

    def tau_at(y):
        if tau_model is not None:
            # the moment bounds grow with depth; a model standing in for them
            # is made non-decreasing along each Gaussian's edges (running
            # maximum: a later edge takes over only when strictly larger)
            tau = tau_model(mom_q, y.reshape(-1)).reshape(y.shape)
            run = [tau[..., 0]]
            for e in range(1, tau.shape[-1]):
                run.append(torch.where(tau[..., e] > run[-1], tau[..., e], run[-1]))
            return torch.stack(run, dim=-1)
        tau, _, _ = bound_tau(mom_q, y.reshape(-1), n_half, opts.beta)
        return tau.reshape(y.shape)

    def warp_y(t):
        return (warp(t, t_near) - centre[slot][:, None]) / scale[slot][:, None]

    if slot.shape[0] > 0:
        q, tau_e, t_e = particle_quadrature(mu, sigma, omega, tau_at, t_near, opts.kappa,
                                            opts.n_intervals, warp_y)
        y_e = warp_y(t_e)
        pen_pair = consistency_penalty(mu, sigma, omega, tau_e, t_e)
    else:
        q = torch.zeros(0, dtype=DT)
        pen_pair = torch.zeros(0, dtype=DT)
        tau_e = y_e = torch.zeros(0, n_edge, dtype=DT)
    penalty = torch.zeros(n_pix, dtype=DT).index_add(0, slot, pen_pair)
    s_rgb = torch.zeros(n_pix, 3, dtype=DT).index_add(0, slot, q[:, None] * rgb_all[gid])
    o = torch.zeros(n_pix, dtype=DT).index_add(0, slot, q)
    image = rescale(mom[:, 0], s_rgb, o, opts.eps, cam.background)
    with torch.no_grad():
        m0 = mom[:, 0].detach()
        live = m0 > 1e-20  # (reading: a pixel below this depth renders background only)
        b = mom.detach() / torch.where(live, m0, torch.ones_like(m0))[:, None]
        b = torch.where(live[:, None], b, _unit_moments(k_mom))
        _, eps = degenerate_mixture(b, n_half)
        fallback = live & (eps != 0)
    return PixelResult(image, s_rgb, o, mom, centre, scale, amb, int(slot.shape[0]),
                       slot, gid, q, y_e, tau_e, penalty, fallback)


def _render_pixels_trig(scene_t, cam, opts, n_pix, slot, gid, amb, mu, sigma, omega, rgb_all,
                        tau_model=None) -> PixelResult:
    """render_pixels with the trigonometric moments of Eqs. 13-14 and the
    bounds on the circle (oracle.trig): the query of an edge at depth t is
    the angle (2 pi - theta) g_hat(t); nothing else changes. ``moments`` holds
    m~_0, then the real and imaginary parts of m~_1..m~_n (K + 1 reals)."""
    if tau_model is not None:
        raise ValueError("the learned surrogate takes power moments")
    n_half = opts.n_moments // 2
    t_near = cam.t_near
    n_edge = opts.n_intervals + 1
    mom_pair = particle_trig_moments(mu, sigma, omega, t_near, n_half)
    mom_c = torch.zeros(n_pix, n_half + 1, dtype=mom_pair.dtype).index_add(0, slot, mom_pair)
    mom_q = mom_c[slot].repeat_interleave(n_edge, dim=0)

    def tau_at(psi):
        tau, _, _ = trig_bound_tau(mom_q, psi.reshape(-1), n_half, opts.beta)
        tau = tau.reshape(psi.shape)
        # non-decreasing along the edges (the circle's estimates need not grow
        # with depth): a later edge takes over only when strictly larger
        run = [tau[..., 0]]
        for e in range(1, tau.shape[-1]):
            run.append(torch.where(tau[..., e] > run[-1], tau[..., e], run[-1]))
        return torch.stack(run, dim=-1)

    def to_angle(t):
        return angle_of(t, t_near)

    if slot.shape[0] > 0:
        q, tau_e, t_e = particle_quadrature(mu, sigma, omega, tau_at, t_near, opts.kappa,
                                            opts.n_intervals, to_angle)
        y_e = to_angle(t_e)
        pen_pair = consistency_penalty(mu, sigma, omega, tau_e, t_e)
        # a pixel with an atom within CUT_BAND of the cut at one of its
        # queries is decided by input rounding (see oracle.trig): ambiguous
        with torch.no_grad():
            marg = cut_margin(mom_q.detach(), y_e.detach().reshape(-1), n_half).reshape(y_e.shape).amin(-1)
            near_cut = torch.zeros(n_pix, dtype=DT).index_add(0, slot, (marg < CUT_BAND).to(DT)) > 0
        amb = amb | near_cut
    else:
        q = torch.zeros(0, dtype=DT)
        pen_pair = torch.zeros(0, dtype=DT)
        tau_e = y_e = torch.zeros(0, n_edge, dtype=DT)
    penalty = torch.zeros(n_pix, dtype=DT).index_add(0, slot, pen_pair)
    s_rgb = torch.zeros(n_pix, 3, dtype=DT).index_add(0, slot, q[:, None] * rgb_all[gid])
    o = torch.zeros(n_pix, dtype=DT).index_add(0, slot, q)
    m0 = mom_c[:, 0].real
    image = rescale(m0, s_rgb, o, opts.eps, cam.background)
    parts = [m0]
    for k in range(1, n_half + 1):
        parts += [mom_c[:, k].real, mom_c[:, k].imag]
    mom = torch.stack(parts, dim=-1)
    with torch.no_grad():
        live = m0.detach() > 1e-20
        unit = torch.zeros_like(mom_c)
        unit[:, 0] = 1.0
        eps = degenerate_flags(torch.where(live[:, None], mom_c.detach(), unit), n_half)
        fallback = live & (eps != 0)
    zeros = torch.zeros(n_pix, dtype=DT)
    return PixelResult(image, s_rgb, o, mom, zeros, zeros + 1.0, amb, int(slot.shape[0]),
                       slot, gid, q, y_e, tau_e, penalty, fallback)


def _unit_moments(k_mom):
    """Standard normal moments (a stand-in for pixels without density)."""
    mom = [1.0, 0.0]
    for j in range(2, k_mom + 1):
        mom.append((j - 1) * mom[j - 2])
    return torch.tensor(mom, dtype=DT)


def _pixel_chunks(cam, px, py, max_pixels):
    for s in range(0, px.shape[0], max_pixels):
        yield s, px[s:s + max_pixels], py[s:s + max_pixels]


def render_image(scene, cam, opts, pixels: Optional[np.ndarray] = None,
                 max_pixels: int = 4096, margin_tol: float = MARGIN_TOL, orient_eps: float = ORIENT_EPS,
                 tau_model=None):
    """Forward render of ``pixels`` (flat indices y * W + x; default: the
    whole image). Returns a dict of numpy arrays: image [P,3], s_rgb [P,3],
    opacity [P], moments [P,K+1], penalty [P] (consistency penalty), ambiguous
    [P] (a coverage decision within ``margin_tol`` pixels of a rectangle edge,
    widened for nearly circular proxies by ``orient_eps``), n_pairs."""
    scene_t = scene_tensors(scene)
    proxy = screen_proxy(scene_t, cam, opts.conf_c)
    if pixels is None:
        pixels = np.arange(cam.width * cam.height)
    pix = torch.as_tensor(np.asarray(pixels), dtype=torch.long)
    px_all, py_all = pix % cam.width, pix // cam.width
    outs = {k: [] for k in ("image", "s_rgb", "opacity", "moments", "centre",
                            "scale", "ambiguous", "penalty", "fallback")}
    n_pairs = 0
    with torch.no_grad():
        for _, px, py in _pixel_chunks(cam, px_all, py_all, max_pixels):
            r = render_pixels(scene_t, scene, cam, opts, px, py, proxy=proxy,
                              margin_tol=margin_tol, orient_eps=orient_eps, tau_model=tau_model)
            outs["image"].append(r.image)
            outs["s_rgb"].append(r.s_rgb)
            outs["opacity"].append(r.opacity)
            outs["moments"].append(r.moments)
            outs["centre"].append(r.centre)
            outs["scale"].append(r.scale)
            outs["ambiguous"].append(r.ambiguous)
            outs["penalty"].append(r.penalty)
            outs["fallback"].append(r.fallback)
            n_pairs += r.n_pairs
    res = {k: torch.cat(v).numpy() for k, v in outs.items()}
    res["n_pairs"] = n_pairs
    return res


def render_backward(scene, cam, opts, grad_image: np.ndarray,
                    pixels: Optional[np.ndarray] = None, max_pixels: int = 2048,
                    grad_penalty: Optional[np.ndarray] = None, tau_model=None):
    """Gradient of sum(grad_image * image) (+ sum(grad_penalty * penalty) when
    given: the per-pixel consistency penalty of App. E) with respect to the scene
    parameters (means, scales, quats, densities, colors), by float64 autograd
    of the forward pass.  Coverage sets and each pixel's moment variable are
    held fixed (the proxy is not differentiated, and the bounds do not depend
    on the moment variable). ``tau_model`` as in ``render_pixels`` (it must be
    differentiable in torch)."""
    scene_t = scene_tensors(scene, requires_grad=True)
    proxy = screen_proxy(scene_t, cam, opts.conf_c)
    if pixels is None:
        pixels = np.arange(cam.width * cam.height)
    pix = torch.as_tensor(np.asarray(pixels), dtype=torch.long)
    px_all, py_all = pix % cam.width, pix // cam.width
    g_img = torch.as_tensor(np.asarray(grad_image), dtype=DT).reshape(-1, 3)
    g_pen = None if grad_penalty is None else torch.as_tensor(np.asarray(grad_penalty), dtype=DT).reshape(-1)
    grads = {k: torch.zeros_like(v) for k, v in scene_t.items()}
    image = []
    for s, px, py in _pixel_chunks(cam, px_all, py_all, max_pixels):
        r = render_pixels(scene_t, scene, cam, opts, px, py, proxy=proxy, tau_model=tau_model)
        loss = (r.image * g_img[s:s + px.shape[0]]).sum()
        if g_pen is not None:
            loss = loss + (r.penalty * g_pen[s:s + px.shape[0]]).sum()
        gs = torch.autograd.grad(loss, [scene_t[k] for k in PARAMS], allow_unused=True)
        for k, g in zip(PARAMS, gs):
            if g is not None:
                grads[k] += g
        image.append(r.image.detach())
    out = {k: v.numpy() for k, v in grads.items()}
    out["image"] = torch.cat(image).numpy()
    return out
