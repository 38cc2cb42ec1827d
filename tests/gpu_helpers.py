"""Shared helpers of the GPU parity tests (HIP path vs CPU oracle)."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
from oracle.proxy import MARGIN_TOL, ORIENT_EPS, screen_proxy
from oracle.render import scene_tensors


def log(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def gpu_render(scene, cams, opts, on_device=False):
    """Forward render through the C ABI. on_device: as the benchmark times
    it, the list count kept on the device (a first frame sizes the capacity,
    the returned second frame has no host round trip), checked to fit."""
    import paper_2512_11800_amd as M
    g = M.Gaussians.from_scene(scene)
    if on_device:
        ws = M.Workspace()
        M.render_forward(g, cams, opts, ws=ws, on_device=True)
        img, saved, st = M.render_forward(g, cams, opts, ws=ws, on_device=True)
        st.check()
    else:
        img, saved, st = M.render_forward(g, cams, opts)
    torch.cuda.synchronize()
    return img.cpu().numpy().astype(np.float64), saved.cpu().numpy().astype(np.float64), st


def proxy_error(scene, cam, opts):
    """Discrepancy between the GPU's rectangles (mb_project: the double
    rectangles its coverage test uses) and the oracle's, over Gaussians both
    keep: centre and half lengths (pixels), the axis angle and the angle times
    the axes' conditioning (1 - minor^2 / major^2), and the count of keep/cull
    disagreements outside the oracle's ambiguous decisions."""
    import paper_2512_11800_amd as M
    g = M.Gaussians.from_scene(scene)
    gp = M.project(g, cam, opts).cpu().numpy()
    op = screen_proxy(scene_tensors(scene), cam, opts.conf_c)
    keep_o = op.valid.numpy()
    amb_o = op.ambiguous.numpy()
    # the GPU also drops a Gaussian whose rectangle's box reaches no pixel centre
    ext = (np.abs(op.axes.numpy()) * op.half.numpy()[:, :, None]).sum(1)
    m2 = op.mean2d.numpy()
    x0 = np.ceil(m2[:, 0] - ext[:, 0] - 0.5)
    x1 = np.floor(m2[:, 0] + ext[:, 0] - 0.5)
    y0 = np.ceil(m2[:, 1] - ext[:, 1] - 0.5)
    y1 = np.floor(m2[:, 1] + ext[:, 1] - 0.5)
    on_screen = ((np.maximum(x0, 0) <= np.minimum(x1, cam.width - 1))
                 & (np.maximum(y0, 0) <= np.minimum(y1, cam.height - 1)))
    near_edge = ((np.abs(x0 - (cam.width - 1)) <= 1) | (np.abs(x1) <= 1)
                 | (np.abs(y0 - (cam.height - 1)) <= 1) | (np.abs(y1) <= 1))
    keep_g = gp[:, 6] > 0
    mismatch = int((keep_o & on_screen & ~near_edge & ~keep_g & ~amb_o).sum()
                   + (keep_g & ~keep_o & ~amb_o).sum())
    both = keep_o & keep_g
    c_err = np.abs(gp[both, :2] - m2[both]).max(initial=0.0)
    h = op.half.numpy()[both]
    h_err = np.abs(gp[both, 4:6] - h).max(initial=0.0)
    eg = gp[both, 2:4]
    eo = op.axes.numpy()[both, 0]
    # sine of the angle between the major axes (either sign)
    sin_a = np.abs(eg[:, 0] * eo[:, 1] - eg[:, 1] * eo[:, 0])
    # the angle error in units of the axes' conditioning, which the band
    # ORIENT_EPS / (1 - minor^2 / major^2) of the protocol is written in
    cond = 1 - (h[:, 1] / h[:, 0]) ** 2
    orient = (sin_a * cond).max(initial=0.0)
    return dict(centre=c_err, half=h_err, angle=sin_a.max(initial=0.0), orient=orient,
                mismatch=mismatch, amb=int(amb_o.sum()), n_keep=int(both.sum()))


def tolerances(pe):
    """The parity protocol's fixed bands (oracle.proxy: MARGIN_TOL pixels at
    rectangle edges, ORIENT_EPS for the axes of near-circles), after checking
    that the measured GPU-oracle rectangle discrepancy sits well inside them."""
    log(f"[proxy] centre {pe['centre']:.2e} half {pe['half']:.2e} angle {pe['angle']:.2e} "
        f"angle x conditioning {pe['orient']:.2e} mismatch {pe['mismatch']} kept {pe['n_keep']}")
    assert pe["mismatch"] == 0
    assert pe["centre"] + pe["half"] <= 0.1 * MARGIN_TOL, pe
    assert pe["orient"] <= 0.1 * ORIENT_EPS, pe
    return MARGIN_TOL, ORIENT_EPS


def compare(img_gpu, res_oracle, label, tol=1e-4, max_excluded=0.0, gpu_saved=None):
    """Per-result max-abs error over pixels the parity protocol keeps. The
    excluded pixels (a coverage or cull decision within the protocol's band;
    with ``gpu_saved`` [P, 8] also pixels whose degenerate-measure flag,
    saved[7] < 0, differs from the oracle's) are counted, logged and bounded:
    at most ``max_excluded`` of the pixels (a fraction; 0 requires none)."""
    ref = res_oracle["image"]
    amb = res_oracle["ambiguous"].copy()
    if gpu_saved is not None:
        flag_gpu = gpu_saved[:, 7] < 0
        disagree = flag_gpu != res_oracle["fallback"]
        log(f"[parity] {label}: degenerate pixels gpu={int(flag_gpu.sum())} "
            f"oracle={int(res_oracle['fallback'].sum())} disagree={int(disagree.sum())}")
        amb |= disagree
    err = np.abs(img_gpu - ref).max(-1)
    keep = ~amb
    mx = float(err[keep].max(initial=0.0))
    p9999 = float(np.quantile(err[keep], 0.9999)) if keep.any() else 0.0
    worst = int(np.argmax(np.where(keep, err, -1)))
    n_ex = int(amb.sum())
    log(f"[parity] {label}: pixels={len(err)} excluded={n_ex} "
        f"max_abs={mx:.3e} p99.99={p9999:.3e} worst_slot={worst} tol={tol:g}")
    assert n_ex <= max_excluded * len(err), f"{label}: {n_ex} of {len(err)} pixels excluded"
    assert np.all(np.isfinite(img_gpu)), f"{label}: non-finite GPU pixels"
    return mx, worst
