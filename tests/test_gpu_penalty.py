"""The consistency penalty of App. E on the GPU: the per-pixel penalty map
against the oracle, and the gradient of a loss with a penalty term against
float64 autograd of the oracle.

Bars: |P_gpu - P_ref| <= 1e-4 max(1, P_ref) per pixel (the penalty is a sum of
squared optical-depth differences, so its float32 error scales with it);
gradients: relative L2 error <= 1e-3 per parameter group, as for the image."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_helpers import log, proxy_error, tolerances
from tests.test_gpu_backward import GROUPS, _rel

pytestmark = pytest.mark.gpu


def _gpu_penalty(scene, cams, opts):
    import paper_2512_11800_amd as M
    g = M.Gaussians.from_scene(scene)
    img, saved, st, pen = M.render_forward(g, cams, opts, penalty=True)
    img2, _, _ = M.render_forward(g, cams, opts)
    torch.cuda.synchronize()
    # the penalty output does not change the image
    assert torch.equal(img, img2)
    return pen.cpu().numpy().astype(np.float64)


def _check_map(pen, ref, keep, label):
    err = np.abs(pen - ref)[keep]
    scale = np.maximum(1.0, ref[keep])
    worst = float((err / scale).max())
    log(f"[penalty] {label}: pixels={keep.sum()} max P={ref.max():.3e} active={(ref > 0).mean():.3f} "
        f"max err/max(1,P)={worst:.3e}")
    assert worst <= 1e-4


@pytest.mark.parametrize("k_mom", [4, 6, 8])
def test_penalty_map_w1(k_mom):
    scene, cams, opts = W.w1_small()
    opts.n_moments = k_mom
    pen = _gpu_penalty(scene, cams, opts)[0].reshape(-1)
    pe = proxy_error(scene, cams[0], opts)
    tol_m, tol_o = tolerances(pe)
    ref = oracle.render_image(scene, cams[0], opts, margin_tol=tol_m, orient_eps=tol_o)
    assert (ref["penalty"] > 0).mean() > 0.05  # the penalty is active on this scene
    _check_map(pen, ref["penalty"], ~ref["ambiguous"], f"W1 K={k_mom}")


def test_penalty_map_w2_sampled():
    from tests.test_gpu_forward import _sample_pixels
    scene, cams, opts = W.w2_clusters()
    cam = cams[0]
    pen = _gpu_penalty(scene, cams, opts)[0].reshape(-1)
    pix = _sample_pixels(scene, cam)
    pe = proxy_error(scene, cam, opts)
    tol_m, tol_o = tolerances(pe)
    ref = oracle.render_image(scene, cam, opts, pixels=pix, margin_tol=tol_m, orient_eps=tol_o)
    _check_map(pen[pix], ref["penalty"], ~ref["ambiguous"], "W2 sampled")


@pytest.mark.parametrize("k_mom", [4, 6])
def test_penalty_gradients_vs_oracle(k_mom):
    """Loss sum(g_img * image) + sum(g_pen * penalty) on the full-coverage
    subset (smooth everywhere)."""
    import paper_2512_11800_amd as M
    scene, cams, opts = W.w3_fd_subset()
    if k_mom == 6:
        scene = scene.subset(np.arange(200))
    opts.n_moments = k_mom
    rng = np.random.default_rng(31 + k_mom)
    g_img = rng.normal(size=(64 * 64, 3))
    g_pen = rng.uniform(0.0, 2.0, size=64 * 64)
    g = M.Gaussians.from_scene(scene)
    img, saved, st, pen = M.render_forward(g, cams, opts, penalty=True)
    gi = torch.as_tensor(g_img, dtype=torch.float32, device="cuda").reshape(img.shape)
    gp = torch.as_tensor(g_pen, dtype=torch.float32, device="cuda").reshape(pen.shape)
    out = M.render_backward(g, cams, opts, st, saved, gi, gp)
    out0 = M.render_backward(g, cams, opts, st, saved, gi)
    torch.cuda.synchronize()
    ref = oracle.render_backward(scene, cams[0], opts, g_img, grad_penalty=g_pen)
    ref0 = oracle.render_backward(scene, cams[0], opts, g_img)
    tol = 1e-3 if k_mom == 4 else 3e-3
    for k in GROUPS:
        a = out[k].cpu().numpy().astype(np.float64)
        r = _rel(a, ref[k])
        # the penalty part alone (difference of the two gradients)
        a_pen = a - out0[k].cpu().numpy().astype(np.float64)
        b_pen = ref[k] - ref0[k]
        r_pen = _rel(a_pen, b_pen) if np.linalg.norm(b_pen) > 0 else 0.0
        log(f"[penalty grad K={k_mom}] {k}: rel_err={r:.3e} penalty part rel_err={r_pen:.3e} "
            f"|penalty part|={np.linalg.norm(b_pen):.3e}")
        assert r <= tol, k
        if k != "colors":  # colours do not enter the penalty
            assert r_pen <= 10 * tol, k


def test_autograd_wrapper_with_penalty():
    import paper_2512_11800_amd as M
    scene, cams, opts = W.w3_fd_subset()
    g = M.Gaussians.from_scene(scene)
    params = [t.clone().requires_grad_(True) for t in (g.means, g.scales, g.quats, g.densities, g.colors)]
    img, pen = M.render(*params, cams, opts, sh_degree=g.sh_degree, with_penalty=True)
    loss = img.square().mean() + 0.1 * pen.mean()
    loss.backward()
    img2, saved, st, pen2 = M.render_forward(g, cams, opts, penalty=True)
    gi = 2.0 * img2 / img2.numel()
    gp = torch.full_like(pen2, 0.1 / pen2.numel())
    ref = M.render_backward(g, cams, opts, st, saved, gi, gp)
    for p, k in zip(params, ("means", "scales", "quats", "densities", "colors")):
        assert torch.allclose(p.grad, ref[k], rtol=1e-5, atol=1e-7), k
