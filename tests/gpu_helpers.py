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
    align = np.abs((gp[both, 2:4] * op.axes.numpy()[both, 0]).sum(-1))
    a_err = np.abs(1 - align).max(initial=0.0)
    h_scale = np.maximum(op.half.numpy()[both].max(-1), 1.0)
    ax_err = (np.sqrt(np.maximum(0, 1 - align ** 2)) * h_scale).max(initial=0.0)
    mismatch = int((keep_o & ~keep_g).sum())
    return dict(centre=c_err, half=h_err, axis=a_err, axis_px=ax_err, mismatch=mismatch,
                amb=int(op.ambiguous.numpy().sum()), n_keep=int(both.sum()))


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
