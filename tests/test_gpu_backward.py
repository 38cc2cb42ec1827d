"""Backward parity: GPU gradients (through the C ABI) against float64 autograd
of the CPU oracle and against central finite differences.

Bar: relative error ||g_gpu - g_ref|| / ||g_ref|| <= 1e-3 per parameter group.
The upstream gradient is a seeded input; pixels whose coverage decision is
ambiguous (parity protocol) get a zero upstream gradient."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_helpers import log, proxy_error, tolerances

pytestmark = pytest.mark.gpu

GROUPS = ("means", "scales", "quats", "densities", "colors")


def _gpu_grads(scene, cams, opts, grad_img, on_device=False):
    """Forward + backward through the C ABI; on_device as the benchmark times
    it (list count on the device, the second frame of a workspace)."""
    import paper_2512_11800_amd as M
    g = M.Gaussians.from_scene(scene)
    ws = M.Workspace()
    if on_device:
        M.render_forward(g, cams, opts, ws=ws, on_device=True)
    img, saved, st = M.render_forward(g, cams, opts, ws=ws, on_device=on_device)
    gi = torch.as_tensor(grad_img, dtype=torch.float32, device="cuda").reshape(img.shape)
    out = M.render_backward(g, cams, opts, st, saved, gi)
    st.check()
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}, img.cpu().numpy()


def _rel(a, b):
    assert np.all(np.isfinite(a)), "non-finite GPU gradient"
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _check(gpu, ref, label, idx=None, tol=1e-3):
    ok = True
    for k in GROUPS:
        a, b = gpu[k], ref[k]
        if idx is not None:
            a, b = a[idx], b[idx]
        r = _rel(a, b)
        log(f"[grad] {label} {k}: rel_err={r:.3e} |ref|={np.linalg.norm(b):.3e}")
        ok = ok and r <= tol
    return ok


def test_fd_subset_vs_oracle_autograd():
    """500 Gaussians of one cluster, 64x64, full coverage (smooth everywhere)."""
    scene, cams, opts = W.w3_fd_subset()
    rng = np.random.default_rng(11)
    g_img = rng.normal(size=(64 * 64, 3))
    gpu, _ = _gpu_grads(scene, cams, opts, g_img)
    ref = oracle.render_backward(scene, cams[0], opts, g_img)
    assert _check(gpu, ref, "fd-subset K=4")


def test_fd_subset_k6_vs_oracle_autograd():
    scene, cams, opts = W.w3_fd_subset()
    scene = scene.subset(np.arange(200))
    opts.n_moments = 6
    rng = np.random.default_rng(12)
    g_img = rng.normal(size=(64 * 64, 3))
    gpu, _ = _gpu_grads(scene, cams, opts, g_img)
    ref = oracle.render_backward(scene, cams[0], opts, g_img)
    assert _check(gpu, ref, "fd-subset K=6", tol=3e-3)


def test_fd_subset_k8_vs_oracle_autograd():
    """Eight moments (the four-atom canonical representation, quartic kernel
    polynomial)."""
    scene, cams, opts = W.w3_fd_subset()
    scene = scene.subset(np.arange(200))
    opts.n_moments = 8
    rng = np.random.default_rng(14)
    g_img = rng.normal(size=(64 * 64, 3))
    gpu, _ = _gpu_grads(scene, cams, opts, g_img)
    ref = oracle.render_backward(scene, cams[0], opts, g_img)
    assert _check(gpu, ref, "fd-subset K=8", tol=3e-3)


@pytest.mark.parametrize("k_mom", [4, 6, 8])
def test_fd_subset_five_intervals_vs_oracle_autograd(k_mom):
    """N = 5 quadrature intervals (six edges per Gaussian)."""
    scene, cams, opts = W.w3_fd_subset()
    scene = scene.subset(np.arange(200))
    opts.n_moments = k_mom
    opts.n_intervals = 5
    rng = np.random.default_rng(20 + k_mom)
    g_img = rng.normal(size=(64 * 64, 3))
    gpu, _ = _gpu_grads(scene, cams, opts, g_img)
    ref = oracle.render_backward(scene, cams[0], opts, g_img)
    assert _check(gpu, ref, f"fd-subset K={k_mom} N=5", tol=3e-3)


def test_w1_proxy_coverage_vs_oracle_autograd():
    """The real proxy coverage (W1); upstream gradient zero on ambiguous pixels."""
    scene, cams, opts = W.w1_small()
    cam = cams[0]
    pe = proxy_error(scene, cam, opts)
    tol_m, tol_o = tolerances(pe)
    amb = oracle.render_image(scene, cam, opts, margin_tol=tol_m, orient_eps=tol_o)["ambiguous"]
    rng = np.random.default_rng(13)
    g_img = rng.normal(size=(cam.width * cam.height, 3))
    g_img[amb] = 0.0
    gpu, _ = _gpu_grads(scene, cams, opts, g_img)
    ref = oracle.render_backward(scene, cam, opts, g_img)
    assert _check(gpu, ref, "W1")


def test_w3_full_size_sampled_gaussians():
    """1M Gaussians at 1600x1064 (the benchmark's training configuration, in
    its launch configuration): gradients of sampled Gaussians, each computed
    by the oracle from every pixel it covers."""
    scene, _, cams, opts = W.w3_train()
    cam = cams[0]
    from oracle.proxy import screen_proxy
    from oracle.render import scene_tensors
    prox = screen_proxy(scene_tensors(scene), cam, opts.conf_c)
    rng = np.random.default_rng(14)
    valid = np.nonzero(prox.valid.numpy())[0]
    # small-footprint Gaussians keep the oracle's pixel set bounded
    area = prox.half.numpy()[valid].prod(-1)
    cand = valid[area < np.quantile(area, 0.5)]
    sample = rng.choice(cand, 12, replace=False)
    pix = set()
    for gi in sample:
        m = prox.mean2d[gi].numpy()
        r = int(np.ceil(prox.half[gi].numpy().sum())) + 1
        xs = np.arange(max(0, int(m[0]) - r), min(cam.width, int(m[0]) + r + 1))
        ys = np.arange(max(0, int(m[1]) - r), min(cam.height, int(m[1]) + r + 1))
        pix.update((yy * cam.width + xx) for yy in ys for xx in xs)
    pix = np.array(sorted(pix))
    pe = proxy_error(scene.subset(sample), cam, opts)
    tol_m, tol_o = tolerances(pe)
    amb = oracle.render_image(scene, cam, opts, pixels=pix, margin_tol=max(tol_m, 1e-3),
                              orient_eps=tol_o)["ambiguous"]
    g_full = np.zeros((cam.width * cam.height, 3))
    vals = rng.normal(size=(len(pix), 3))
    vals[amb] = 0.0
    g_full[pix] = vals
    gpu, _ = _gpu_grads(scene, cams, opts, g_full, on_device=True)
    ref = oracle.render_backward(scene, cam, opts, vals, pixels=pix)
    log(f"[w3] sampled {len(sample)} Gaussians over {len(pix)} pixels ({int(amb.sum())} ambiguous)")
    assert _check(gpu, ref, "W3 sampled", idx=sample, tol=2e-3)


def test_gpu_finite_differences():
    """Central differences of the GPU's own float32 forward (coarse steps)."""
    import paper_2512_11800_amd as M
    scene, cams, opts = W.w3_fd_subset()
    scene = scene.subset(np.arange(60))
    rng = np.random.default_rng(15)
    g_img = rng.normal(size=(64 * 64, 3))
    gpu, _ = _gpu_grads(scene, cams, opts, g_img)

    def loss(sc):
        g = M.Gaussians.from_scene(sc)
        img, _, _ = M.render_forward(g, cams, opts)
        img = img.double().cpu().numpy().reshape(-1, 3)
        assert np.all(np.isfinite(img))
        return float((img * g_img).sum())

    worst = 0.0
    for name, h in (("means", 1e-3), ("scales", 2e-4), ("densities", 1e-2), ("colors", 1e-2)):
        arr = getattr(scene, name)
        for _ in range(3):
            idx = tuple(rng.integers(0, s) for s in arr.shape)
            sp = scene.copy()
            getattr(sp, name)[idx] += h
            sm = scene.copy()
            getattr(sm, name)[idx] -= h
            fd = (loss(sp) - loss(sm)) / (2 * h)
            an = gpu[name][idx]
            assert np.isfinite(fd) and np.isfinite(an)
            err = abs(fd - an) / max(abs(fd), abs(an), 1e-3)
            worst = max(worst, err)
            log(f"[fd] {name}{idx}: fd={fd:.5e} analytic={an:.5e} rel={err:.2e}")
    assert worst < 5e-2


def test_autograd_wrapper_matches_direct_call():
    import paper_2512_11800_amd as M
    scene, cams, opts = W.w1_small()
    dev = "cuda"
    params = {k: torch.tensor(getattr(scene, k), device=dev, requires_grad=True) for k in GROUPS}
    img = M.render(params["means"], params["scales"], params["quats"], params["densities"],
                   params["colors"], cams, opts, sh_degree=scene.sh_degree)
    w = torch.randn_like(img)
    (img * w).sum().backward()
    direct, _ = _gpu_grads(scene, cams, opts, w.cpu().numpy().reshape(-1, 3))
    for k in GROUPS:
        assert np.allclose(params[k].grad.cpu().numpy(), direct[k], rtol=1e-6, atol=1e-9), k
