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


def gpu_render(scene, cams, opts):
    import paper_2512_11800_amd as M
    g = M.Gaussians.from_scene(scene)
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
    keep_g = gp[:, 6] > 0
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
    mismatch = int((keep_o & ~keep_g).sum())
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
