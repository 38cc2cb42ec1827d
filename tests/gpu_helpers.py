"""Shared helpers of the GPU parity tests (HIP path vs CPU oracle)."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
from oracle.proxy import screen_proxy
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
    """Max discrepancy (pixels) between the GPU and oracle proxy rectangles over
    Gaussians both keep, and the count of keep/cull disagreements."""
    import paper_2512_11800_amd as M
    g = M.Gaussians.from_scene(scene)
    gp = M.project(g, cam, opts).cpu().numpy().astype(np.float64)
    op = screen_proxy(scene_tensors(scene), cam, opts.conf_c)
    keep_o = op.valid.numpy()
    # the GPU keeps a Gaussian only if its rectangle's box reaches a pixel centre
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
    amb_o = op.ambiguous.numpy()
    # decisions that must agree: clearly on screen, or culled by the oracle
    mismatch_n = int((keep_o & on_screen & ~near_edge & ~keep_g & ~amb_o).sum()
                     + (keep_g & ~keep_o & ~amb_o).sum())
    # the GPU also drops Gaussians whose rectangle misses the image
    both = keep_o & keep_g
    c_err = np.abs(gp[both, :2] - op.mean2d.numpy()[both]).max(initial=0.0)
    h_err = np.abs(gp[both, 4:6] - op.half.numpy()[both]).max(initial=0.0)
    eg = gp[both, 2:4]
    eo = op.axes.numpy()[both, 0]
    # sine of the angle between the axes from the cross product (accurate for
    # small angles, unlike sqrt(1 - cos^2) of float32 unit vectors)
    angle = np.abs(eg[:, 0] * eo[:, 1] - eg[:, 1] * eo[:, 0]) / (
        np.linalg.norm(eg, axis=1) * np.linalg.norm(eo, axis=1))
    h = op.half.numpy()[both]
    # axis angle error relative to the conditioning of the eigenvectors
    orient = (angle * (1 - (h[:, 0] / np.maximum(h[:, 1], 1e-300)) ** 2)).max(initial=0.0)
    mismatch = mismatch_n
    return dict(centre=c_err, half=h_err, orient=orient, angle=angle.max(initial=0.0),
                mismatch=mismatch, amb=int(op.ambiguous.numpy().sum()), n_keep=int(both.sum()))


def tolerances(pe):
    """Exclusion band for the parity protocol from the measured proxy
    discrepancy: (margin in pixels, orientation epsilon)."""
    return max(1e-4, 4.0 * (pe["centre"] + pe["half"])), max(1e-6, 4.0 * pe["orient"])


def compare(img_gpu, res_oracle, label, tol=1e-4):
    """Per-result max-abs error over pixels the parity protocol keeps."""
    ref = res_oracle["image"]
    amb = res_oracle["ambiguous"]
    err = np.abs(img_gpu - ref).max(-1)
    keep = ~amb
    mx = float(err[keep].max(initial=0.0))
    p9999 = float(np.quantile(err[keep], 0.9999)) if keep.any() else 0.0
    worst = int(np.argmax(np.where(keep, err, -1)))
    log(f"[parity] {label}: pixels={len(err)} excluded={int(amb.sum())} "
        f"max_abs={mx:.3e} p99.99={p9999:.3e} worst_slot={worst} tol={tol:g}")
    return mx, worst
