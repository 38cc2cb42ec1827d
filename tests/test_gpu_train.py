"""The training-system pieces together: fit a perturbed copy of a scene back
to renders of the original with the paper's objective (L1, D-SSIM and the
consistency penalty), Adam on the means and colours, then one
adaptive-density-control step and more training of the new set. Property
bars: the objective falls by a third and the render's PSNR against the
target rises (single-view fitting does not pin individual positions, so
their error is only logged); the densified set has the planned size, renders
finite, and training it (fresh optimiser state) at least halves its L1. The
first fit runs its frames with the list count on the device (no host round
trip per step), each checked to fit its workspace; the second takes counts."""
import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu


def test_fit_a_perturbed_scene_then_densify():
    import paper_2512_11800_amd as M
    from paper_2512_11800_amd import adc as ADC
    from paper_2512_11800_amd import loss as GL
    from paper_2512_11800_amd import train as T
    scene, cams, opts = W.w1_small()
    opts.n_moments = 4
    ref = M.Gaussians.from_scene(scene)
    target, _, _ = M.render_forward(ref, cams, opts)
    target = target.clone()
    rng = np.random.default_rng(0)
    moved = scene.subset(np.arange(scene.n))
    moved.means = (scene.means + rng.normal(0, 0.02, scene.means.shape)).astype(np.float32)
    g = M.Gaussians.from_scene(moved)
    err0 = float((g.means - ref.means).norm(dim=1).mean())
    img0, _, _ = M.render_forward(g, cams, opts)
    psnr0 = float(-10 * torch.log10(((img0 - target) ** 2).mean()))
    adam = T.Adam({"means": 2e-3, "colors": 5e-3})
    state = ADC.AdcState.zeros(g.n)
    first = None
    ws = M.Workspace()
    for it in range(60):  # frames with the list count on the device, checked every step
        terms = T.train_step(g, cams, opts, target, adam, state, ws=ws, on_device=True)
        terms["state"].check()
        tot = float(terms["total"])
        first = tot if first is None else first
        if it % 20 == 0:
            log(f"[train] step {it}: total {tot:.5f} l1 {float(terms['l1']):.5f} "
                f"dssim {float(terms['dssim']):.5f} consistency {float(terms['consistency']):.3e}")
    err1 = float((g.means - ref.means).norm(dim=1).mean())
    img1, _, _ = M.render_forward(g, cams, opts)
    psnr1 = float(-10 * torch.log10(((img1 - target) ** 2).mean()))
    log(f"[train] objective {first:.5f} -> {tot:.5f}; PSNR vs target {psnr0:.2f} -> {psnr1:.2f} dB; "
        f"mean position error {err0:.4f} -> {err1:.4f}")
    assert tot < 0.67 * first
    assert psnr1 > psnr0 + 3.0
    # one density-control step: every action occurs at these thresholds
    action, offsets, n_out = ADC.plan(g, state, min_opacity=0.01, grad_threshold=2e-5,
                                      split_scale=float(g.scales.max(dim=1).values.median()))
    counts = np.bincount(action.cpu().numpy(), minlength=4)
    g2 = ADC.apply(g, action, offsets, n_out)
    img2, _, _ = M.render_forward(g2, cams, opts)
    l1b = float(GL.l1(img2, target))
    log(f"[train] density control: {counts} (prune, keep, clone, split) -> {g2.n} particles; "
        f"L1 {float(terms['l1']):.5f} -> {l1b:.5f}")
    assert torch.isfinite(img2).all()
    assert g2.n == n_out == counts[1] + 2 * (counts[2] + counts[3])
    adam2 = T.Adam({"means": 2e-3, "colors": 5e-3})
    for _ in range(40):
        terms2 = T.train_step(g2, cams, opts, target, adam2)
    l1c = float(terms2["l1"])
    log(f"[train] after 40 more steps on the densified set: L1 {l1c:.5f}")
    assert l1c < 0.5 * l1b
