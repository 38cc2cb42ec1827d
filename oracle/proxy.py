"""Frustum culling and the confidence-interval screen proxy (float64).

TEST INFRASTRUCTURE: see the package docstring.

Sec. 3.3 (Eqs. 16-21) and App. D: a Gaussian is rasterised as the oriented
bounding rectangle of the screen-space ellipse on which its isolated opacity
1 - exp(-tau_bar) equals the confidence level c, with tau_bar replaced by the
erf-free form and Sigma approximated along the view vector.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from .geometry import DT


@dataclass
class Proxy:
    mean2d: torch.Tensor     # [n,2] ellipse centre (pixels)
    axes: torch.Tensor       # [n,2,2] rows: unit eigenvectors e_1, e_2 of Sigma_2d
    half: torch.Tensor       # [n,2] half side lengths sqrt(lambda_k)
    valid: torch.Tensor      # [n] bool: not culled and a real ellipse
    ambiguous: torch.Tensor  # [n] bool: a cull/ellipse decision is within rounding
    kappa: torch.Tensor      # [n]
    quad: torch.Tensor       # [n] mean^T A mean (camera frame)
    in_frustum: torch.Tensor  # [n] bool: the bounding-sphere cull alone keeps it


# Bands of the parity protocol for decisions taken at a threshold. The HIP
# path takes every per-Gaussian decision (cull, proxy, rectangle) in double
# precision from the same float32 inputs, so the two sides can differ only by
# double rounding: relative 1e-12 is thousands of times that.
CULL_REL = 1e-12
# Coverage decisions (pixel centre against rectangle edge): the HIP path tests
# in double against a rectangle computed in double in a cancellation-free
# form; the long-double homogeneous conic here still loses up to ten digits
# for distant elongated Gaussians (measured against the cancellation-free form
# in long double: 5e-9 px on the half lengths of the 500k-Gaussian 1080p frame,
# 1.2e-7 px at 3M Gaussians and 4K). So |margin| < MARGIN_TOL pixels is
# ambiguous, and the axes of a near-circle are ambiguous to
# ORIENT_EPS / (1 - minor^2 / major^2) radians (their conditioning).
MARGIN_TOL = 2e-6
ORIENT_EPS = 1e-11


def _quat_rot_ld(q: np.ndarray) -> np.ndarray:
    """Rotation matrices [n,3,3] of quaternions (w, x, y, z), normalised first
    (the Sec. 3.1 parameterisation), in numpy long double."""
    q = q / np.sqrt((q * q).sum(-1, keepdims=True))
    w, x, y, z = q.T
    r = np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                  2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                  2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)
    return r.reshape(-1, 3, 3)


def screen_proxy(scene_t, cam, conf_c: float) -> Proxy:
    """Per-Gaussian culling and proxy.

    Culling (Sec. 3.3): the bounding sphere (mean, r = max diag S) is tested
    against the near plane z = t_n and the four side planes; the centre must
    also lie beyond the near plane, and the proxy must be a real ellipse
    (App. D: 0 < kappa < mean^T A mean, W_2x2 negative definite).

    Proxy (Eqs. 17-21, App. D), in camera coordinates with A = Sigma^-1:
        C     = -log(1 - c) sqrt(u^T A u) / sqrt(2 pi),  u = mean / |mean|
        kappa = 2 (log C - log w) + mean^T A mean
        m = K^-T A mean,  M = K^-T A K^-1,  W = m m^T - kappa M
        mean2d = -W22^-1 w21,  Sigma2d = (mean2d^T W22 mean2d - w33) W22^-1
    and the rectangle spans sqrt(lambda_k) e_k over the eigenpairs of Sigma2d.

    The paper names the oriented box of the ellipse but not its orientation
    when the ellipse is (nearly) a circle, where the eigenvectors are
    ill-conditioned. Reading: the first axis is the major axis at the angle
    theta = atan2(2 s_xy, s_xx - s_yy) / 2 of Sigma2d = [[s_xx, s_xy],
    [s_xy, s_yy]], the second axis is it turned by +90 degrees, and an exact
    circle (s_xy = 0, s_xx = s_yy) takes theta = atan2(0, 0) / 2 = 0.

    The homogeneous conic cancels: m m^T and kappa M agree in their leading
    digits, so float64 loses about seven of them (3e-7 px on the half lengths
    of 1080p proxies). The formulas are therefore evaluated as written in
    numpy long double (64-bit mantissa on x86) from the float32 inputs; the
    results are returned as float64 tensors. Nothing here is differentiated.
    """
    LD = np.longdouble
    w2c = np.asarray(cam.world_to_cam).astype(LD)
    r_wc, t_wc = w2c[:, :3], w2c[:, 3]
    means, scales, quats, dens = (scene_t[k].detach().numpy().astype(LD) for k in
                                  ("means", "scales", "quats", "densities"))
    fx, fy, cx, cy, t_near = (LD(v) for v in (cam.fx, cam.fy, cam.cx, cam.cy, cam.t_near))
    mu_c = means @ r_wc.T + t_wc
    rot_c = r_wc @ _quat_rot_ld(quats)
    a = (rot_c / (scales ** 2)[:, None, :]) @ np.swapaxes(rot_c, -1, -2)

    # --- culling with the bounding sphere -----------------------------------
    radius = scales.max(axis=-1)
    w_img, h_img = LD(cam.width), LD(cam.height)
    normals = np.array([[fx, 0, cx], [-fx, 0, w_img - cx],
                        [0, fy, cy], [0, -fy, h_img - cy]], dtype=LD)
    normals = normals / np.sqrt((normals ** 2).sum(-1, keepdims=True))
    side = mu_c @ normals.T + radius[:, None]           # >= 0: not wholly outside
    near_sphere = mu_c[:, 2] + radius - t_near           # >= 0: not wholly in front of t_n
    near_centre = mu_c[:, 2] - t_near                   # > 0 required
    in_frustum = (side >= 0).all(-1) & (near_sphere >= 0) & (near_centre > 0)

    # --- confidence-interval conic -------------------------------------------
    norm_c = np.sqrt((mu_c ** 2).sum(-1))
    u = mu_c / norm_c[:, None]
    uau = np.einsum("ni,nij,nj->n", u, a, u)
    big_c = -np.log1p(-LD(conf_c)) * np.sqrt(uau) / np.sqrt(2 * LD(np.pi))
    quad = np.einsum("ni,nij,nj->n", mu_c, a, mu_c)
    with np.errstate(divide="ignore"):
        kappa = 2 * (np.log(big_c) - np.log(dens)) + quad
    kinv = np.array([[1 / fx, 0, -cx / fx], [0, 1 / fy, -cy / fy], [0, 0, 1]], dtype=LD)
    m = (kinv.T @ (a @ mu_c[:, :, None]))[:, :, 0]
    big_m = kinv.T @ a @ kinv
    w = m[:, :, None] * m[:, None, :] - kappa[:, None, None] * big_m
    w22 = w[:, :2, :2]
    w21 = w[:, :2, 2]
    w33 = w[:, 2, 2]
    # W22 negative definite <=> trace < 0 and det > 0
    det22 = w22[:, 0, 0] * w22[:, 1, 1] - w22[:, 0, 1] * w22[:, 1, 0]
    tr22 = w22[:, 0, 0] + w22[:, 1, 1]
    ell_ok = (kappa > 0) & (kappa < quad) & (det22 > 0) & (tr22 < 0)
    d_safe = np.where(ell_ok, det22, 1)
    w22_inv = np.stack([np.stack([w22[:, 1, 1], -w22[:, 0, 1]], -1),
                        np.stack([-w22[:, 1, 0], w22[:, 0, 0]], -1)], -2) / d_safe[:, None, None]
    mean2d = -(w22_inv @ w21[:, :, None])[:, :, 0]
    s2 = np.einsum("ni,nij,nj->n", mean2d, w22, mean2d) - w33
    ell_ok = ell_ok & (s2 < 0)
    sigma2d = s2[:, None, None] * w22_inv
    sigma2d = np.where(ell_ok[:, None, None], sigma2d, np.eye(2, dtype=LD))
    sxx, syy, sxy = sigma2d[:, 0, 0], sigma2d[:, 1, 1], sigma2d[:, 0, 1]
    theta = np.arctan2(2 * sxy, sxx - syy) / 2
    mid = (sxx + syy) / 2
    rad = np.sqrt(((sxx - syy) / 2) ** 2 + sxy ** 2)
    lam_major = mid + rad
    lam_minor = (sxx * syy - sxy * sxy) / lam_major  # mid - rad without cancellation
    half = np.sqrt(np.clip(np.stack([lam_major, lam_minor], -1), 0, None))
    c_t, s_t = np.cos(theta), np.sin(theta)
    axes = np.stack([np.stack([c_t, s_t], -1), np.stack([-s_t, c_t], -1)], -2)  # rows e_1, e_2

    valid = in_frustum & ell_ok
    # decisions within double rounding of their threshold (both sides decide
    # in double or better from the same float32 inputs)
    scale_side = norm_c[:, None] + radius[:, None]
    amb = ((np.abs(side) < CULL_REL * scale_side).any(-1)
           | (np.abs(near_sphere) < CULL_REL * (1 + norm_c + radius))
           | (np.abs(near_centre) < CULL_REL * (1 + norm_c))
           | (np.abs(quad - kappa) < CULL_REL * (1 + quad + np.abs(kappa)))
           | (np.abs(kappa) < CULL_REL * (1 + quad)))

    def t64(x):
        return torch.from_numpy(np.asarray(x, dtype=np.float64))

    return Proxy(t64(mean2d), t64(axes), t64(half), torch.from_numpy(valid), torch.from_numpy(amb),
                 t64(kappa), t64(quad), torch.from_numpy(in_frustum))


def rect_margin(proxy: Proxy, gidx: torch.Tensor, px: torch.Tensor, py: torch.Tensor):
    """Signed distance (pixels) of the pixel centre inside the oriented
    rectangle: min_k (sqrt(lambda_k) - |(p - mean2d) . e_k|); >= 0 covers."""
    p = torch.stack([px.to(DT) + 0.5, py.to(DT) + 0.5], dim=-1) - proxy.mean2d[gidx]
    proj = (proxy.axes[gidx] @ p.unsqueeze(-1)).squeeze(-1).abs()
    return (proxy.half[gidx] - proj).min(dim=-1).values


def _decision_tol(proxy: Proxy, gidx, px, py, margin_tol, orient_eps):
    """Per-pair width of the band of ambiguous coverage decisions: a fixed
    margin plus the motion of the rectangle's edges under a rotation of its
    axes by orient_eps / (1 - lambda_1/lambda_2) (the axes of a nearly circular
    ellipse are ill-conditioned; for a circle every orientation is valid)."""
    if orient_eps <= 0:
        return margin_tol
    h = proxy.half[gidx]
    ratio = (h[:, 1] / h[:, 0].clamp_min(1e-300)) ** 2  # minor / major
    dtheta = (orient_eps / (1 - ratio).clamp_min(1e-300)).clamp_max(math.pi)
    p = torch.stack([px.to(DT) + 0.5, py.to(DT) + 0.5], dim=-1) - proxy.mean2d[gidx]
    return margin_tol + dtheta * p.norm(dim=-1)


def covering_pairs(proxy: Proxy, cam, pix_x: torch.Tensor, pix_y: torch.Tensor,
                   margin_tol: float = MARGIN_TOL, full_coverage: bool = False,
                   chunk: int = 1 << 22, orient_eps: float = ORIENT_EPS):
    """Pairs (pixel slot, Gaussian) with the pixel centre inside the Gaussian's
    rectangle (the proxy the paper rasterises; App. D).

    ``pix_x``/``pix_y`` list the pixels to evaluate (slot = position in the
    list). Also returns a per-slot flag for pixels where some coverage
    decision is within ``margin_tol`` pixels of a rectangle edge or the
    Gaussian's cull decision is within rounding (the parity protocol excludes
    those)."""
    n_pix = pix_x.shape[0]
    n_g = proxy.valid.shape[0]
    if full_coverage:
        slot = torch.arange(n_pix).repeat_interleave(n_g)
        gid = torch.arange(n_g).repeat(n_pix)
        return slot, gid, torch.zeros(n_pix, dtype=torch.bool)
    g_ok = torch.nonzero(proxy.valid | proxy.ambiguous).squeeze(-1)
    # axis-aligned extent of each rectangle, dilated by the tolerance
    ext = (proxy.axes[g_ok].abs() * proxy.half[g_ok][:, :, None]).sum(1) + margin_tol
    if orient_eps > 0:
        # room for the band of a rotated rectangle around its corners
        h = proxy.half[g_ok]
        ratio = (h[:, 1] / h[:, 0].clamp_min(1e-300)) ** 2  # minor / major
        dtheta = (orient_eps / (1 - ratio).clamp_min(1e-300)).clamp_max(math.pi)
        ext = ext + (dtheta * (h[:, 0] + h[:, 1]))[:, None]
    lo = proxy.mean2d[g_ok] - ext
    hi = proxy.mean2d[g_ok] + ext
    if n_pix <= 4096:
        return _pairs_by_pixel(proxy, g_ok, lo, hi, pix_x, pix_y, margin_tol, n_g, orient_eps)
    # candidate pixels of each Gaussian: those in the pixel list whose centre
    # lies in its dilated box; a dense lookup from image position to slot.
    slot_of = torch.full((cam.height, cam.width), -1, dtype=torch.long)
    slot_of[pix_y, pix_x] = torch.arange(n_pix)
    x0 = torch.ceil(lo[:, 0] - 0.5).clamp(0, cam.width - 1).long()
    x1 = torch.floor(hi[:, 0] - 0.5).clamp(-1, cam.width - 1).long()
    y0 = torch.ceil(lo[:, 1] - 0.5).clamp(0, cam.height - 1).long()
    y1 = torch.floor(hi[:, 1] - 0.5).clamp(-1, cam.height - 1).long()
    nx = (x1 - x0 + 1).clamp_min(0)
    ny = (y1 - y0 + 1).clamp_min(0)
    cnt = nx * ny
    slots, gids, amb_slots = [], [], []
    # enumerate boxes in chunks of Gaussians whose total box area fits `chunk`
    csum = torch.cumsum(cnt, 0)
    start = 0
    while start < g_ok.shape[0]:
        base = csum[start - 1] if start > 0 else torch.tensor(0)
        stop = int(torch.searchsorted(csum, base + chunk, right=True))
        stop = max(stop, start + 1)
        sel = torch.arange(start, stop)
        c = cnt[sel]
        total = int(c.sum())
        if total > 0:
            owner = sel.repeat_interleave(c)
            first = torch.cumsum(c, 0) - c
            local = torch.arange(total) - first.repeat_interleave(c)
            xx = x0[owner] + local % nx[owner]
            yy = y0[owner] + local // nx[owner]
            sl = slot_of[yy, xx]
            keep = sl >= 0
            owner, xx, yy, sl = owner[keep], xx[keep], yy[keep], sl[keep]
            g = g_ok[owner]
            marg = rect_margin(proxy, g, xx, yy)
            cov = (marg >= 0) & proxy.valid[g]
            slots.append(sl[cov])
            gids.append(g[cov])
            tol = _decision_tol(proxy, g, xx, yy, margin_tol, orient_eps)
            amb = (marg.abs() < tol) | (proxy.ambiguous[g] & (marg >= -tol))
            amb_slots.append(sl[amb])
        start = stop
    slot = torch.cat(slots) if slots else torch.zeros(0, dtype=torch.long)
    gid = torch.cat(gids) if gids else torch.zeros(0, dtype=torch.long)
    # order by (slot, gid)
    order = torch.argsort(slot * n_g + gid)
    ambiguous = torch.zeros(n_pix, dtype=torch.bool)
    if amb_slots:
        a = torch.cat(amb_slots)
        ambiguous[a] = True
    return slot[order], gid[order], ambiguous


def _pairs_by_pixel(proxy, g_ok, lo, hi, pix_x, pix_y, margin_tol, n_g, orient_eps):
    """Same pairs as ``covering_pairs`` for a short pixel list: each pixel is
    tested against every Gaussian whose dilated box contains its centre."""
    slots, gids, ambiguous = [], [], torch.zeros(pix_x.shape[0], dtype=torch.bool)
    for s in range(pix_x.shape[0]):
        u = float(pix_x[s]) + 0.5
        v = float(pix_y[s]) + 0.5
        cand = g_ok[(lo[:, 0] <= u) & (hi[:, 0] >= u) & (lo[:, 1] <= v) & (hi[:, 1] >= v)]
        if cand.numel() == 0:
            continue
        xs = pix_x[s].expand(cand.shape[0])
        ys = pix_y[s].expand(cand.shape[0])
        marg = rect_margin(proxy, cand, xs, ys)
        cov = (marg >= 0) & proxy.valid[cand]
        slots.append(torch.full((int(cov.sum()),), s, dtype=torch.long))
        gids.append(cand[cov])
        tol = _decision_tol(proxy, cand, xs, ys, margin_tol, orient_eps)
        if bool(((marg.abs() < tol) | (proxy.ambiguous[cand] & (marg >= -tol))).any()):
            ambiguous[s] = True
    slot = torch.cat(slots) if slots else torch.zeros(0, dtype=torch.long)
    gid = torch.cat(gids) if gids else torch.zeros(0, dtype=torch.long)
    order = torch.argsort(slot * n_g + gid)
    return slot[order], gid[order], ambiguous
