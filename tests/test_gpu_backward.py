"""Backward parity: GPU gradients (through the C ABI) against float64 autograd
of the CPU oracle and against central finite differences.

Bar, per parameter group: relative error ||g_gpu - g_ref|| / ||g_ref|| <= 1e-3,
and element by element max |g_gpu - g_ref| <= 1e-3 max |g_ref| (so a few wrong
Gaussians cannot hide in the group norm). The upstream gradient is a seeded
input; pixels whose coverage decision is ambiguous (parity protocol) get a
zero upstream gradient."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from oracle.proxy import screen_proxy
from oracle.render import scene_tensors
from tests.gpu_helpers import gpu_render, log, proxy_error, tolerances

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


def _check(gpu, ref, label, idx=None, ref_idx=None, tol=1e-3):
    ok = True
    for k in GROUPS:
        a, b = gpu[k], ref[k]
        if idx is not None:
            a = a[idx]
            b = b[idx if ref_idx is None else ref_idx]
        r = _rel(a, b)
        el = float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))
        log(f"[grad] {label} {k}: rel_err={r:.3e} max_elem_err/max|ref|={el:.3e} "
            f"|ref|={np.linalg.norm(b):.3e}")
        ok = ok and r <= tol and el <= tol
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
    assert _check(gpu, ref, "fd-subset K=6")


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
    assert _check(gpu, ref, "fd-subset K=8")


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
    assert _check(gpu, ref, f"fd-subset K={k_mom} N=5")


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


@pytest.mark.parametrize("k_mom,basis", [(4, "power"), (6, "power"), (8, "power"), (4, "trigonometric")])
def test_w3_full_size_sampled_gaussians(k_mom, basis):
    """1M Gaussians at 1600x1064 (the benchmark's training configuration, in
    its launch configuration): gradients of sampled Gaussians, each computed by
    the oracle from every pixel its rectangle's box reaches. The sample mixes
    small footprints (below the median area), large ones (median to 95th
    percentile) and Gaussians in the heaviest tiles, whose lists are long
    enough to be rendered split over four workgroups. The oracle renders only
    the Gaussians whose box reaches a sampled pixel: the others change no
    sampled pixel."""
    scene, _, cams, opts = W.w3_train()
    opts.n_moments = k_mom
    opts.basis = basis
    cam = cams[0]
    prox = screen_proxy(scene_tensors(scene), cam, opts.conf_c)
    rng = np.random.default_rng(14 + k_mom)
    lo, hi = _boxes(prox, cam)
    valid = np.nonzero(prox.valid.numpy())[0]
    area = prox.half.numpy()[valid].prod(-1)
    q50, q95 = np.quantile(area, [0.5, 0.95])
    small = valid[area < q50]
    large = valid[(area >= q50) & (area < q95)]
    # tile list lengths from the boxes (an upper bound of the lists)
    tiles_x, tiles_y = (cam.width + 15) // 16, (cam.height + 15) // 16
    cnt = np.zeros((tiles_y + 1, tiles_x + 1), np.int64)
    t0 = np.clip(lo[valid] // 16, 0, [tiles_x - 1, tiles_y - 1]).astype(int)
    t1 = np.clip(hi[valid] // 16, 0, [tiles_x - 1, tiles_y - 1]).astype(int)
    np.add.at(cnt, (t0[:, 1], t0[:, 0]), 1)
    np.add.at(cnt, (t0[:, 1], t1[:, 0] + 1), -1)
    np.add.at(cnt, (t1[:, 1] + 1, t0[:, 0]), -1)
    np.add.at(cnt, (t1[:, 1] + 1, t1[:, 0] + 1), 1)
    cnt = cnt.cumsum(0).cumsum(1)[:tiles_y, :tiles_x]
    heavy_t = np.argsort(cnt.ravel())[::-1][:8]
    log(f"[w3] heaviest tiles hold up to {cnt.ravel()[heavy_t].max()} / {cnt.ravel()[heavy_t].min()} box entries")
    hty, htx = heavy_t // tiles_x, heavy_t % tiles_x
    in_heavy = np.zeros(len(valid), bool)
    for yy, xx in zip(hty, htx):
        in_heavy |= ((t0[:, 0] <= xx) & (t1[:, 0] >= xx) & (t0[:, 1] <= yy) & (t1[:, 1] >= yy))
    heavy = valid[in_heavy & (area < q95)]
    sample = np.unique(np.concatenate([rng.choice(small, 5, replace=False),
                                       rng.choice(large, 5, replace=False),
                                       rng.choice(heavy, 5, replace=False)]))
    pix = set()
    for gi in sample:
        xs = np.arange(max(0, int(np.floor(lo[gi, 0]))), min(cam.width, int(np.ceil(hi[gi, 0])) + 1))
        ys = np.arange(max(0, int(np.floor(lo[gi, 1]))), min(cam.height, int(np.ceil(hi[gi, 1])) + 1))
        pix.update((yy * cam.width + xx) for yy in ys for xx in xs)
    pix = np.array(sorted(pix))
    tol_m, tol_o = tolerances(proxy_error(scene.subset(sample), cam, opts))
    sub = _touching(prox, lo, hi, cam, pix)
    assert np.isin(sample, sub).all()
    sub_scene = scene.subset(sub)
    ref_img = oracle.render_image(sub_scene, cam, opts, pixels=pix, margin_tol=tol_m, orient_eps=tol_o,
                                  max_pixels=len(pix))
    # no upstream gradient where the coverage decision is ambiguous or the
    # degenerate-measure flags of the two sides differ; for the trigonometric
    # moments the ambiguous pixels also hold those with an atom of the
    # reconstruction at the circle's cut (oracle.trig.CUT_BAND), bounded as in
    # the trigonometric image tests
    _, saved, _ = gpu_render(scene, cams, opts, on_device=True)
    flag_gpu = saved[0].reshape(-1, 8)[pix, 7] < 0
    amb = ref_img["ambiguous"] | (flag_gpu != ref_img["fallback"])
    assert amb.sum() <= (0.02 if basis == "trigonometric" else 0.01) * len(pix)
    g_full = np.zeros((cam.width * cam.height, 3))
    vals = rng.normal(size=(len(pix), 3))
    vals[amb] = 0.0
    g_full[pix] = vals
    gpu, _ = _gpu_grads(scene, cams, opts, g_full, on_device=True)
    ref = oracle.render_backward(sub_scene, cam, opts, vals, pixels=pix, max_pixels=len(pix))
    log(f"[w3 K={k_mom} {basis}] sampled {len(sample)} Gaussians over {len(pix)} pixels "
        f"({int(amb.sum())} ambiguous), oracle scene {len(sub)} Gaussians")
    assert _check(gpu, ref, f"W3 K={k_mom} {basis} sampled", idx=sample, ref_idx=np.searchsorted(sub, sample))


def _boxes(prox, cam):
    """Axis-aligned pixel-centre boxes [lo, hi] of the oracle's rectangles."""
    ext = (np.abs(prox.axes.numpy()) * prox.half.numpy()[:, :, None]).sum(1) + 1e-3
    m = prox.mean2d.numpy()
    return m - ext - 0.5, m + ext - 0.5


def _touching(prox, lo, hi, cam, pix):
    """Indices of the Gaussians (kept or ambiguous) whose box holds a pixel of
    `pix` (flat y * W + x), through a summed-area table of the pixel set."""
    ind = np.zeros((cam.height + 1, cam.width + 1), np.int64)
    ind[1:, 1:][pix // cam.width, pix % cam.width] = 1
    sat = ind.cumsum(0).cumsum(1)
    x0 = np.clip(np.ceil(lo[:, 0]), 0, cam.width).astype(int)
    x1 = np.clip(np.floor(hi[:, 0]) + 1, 0, cam.width).astype(int)
    y0 = np.clip(np.ceil(lo[:, 1]), 0, cam.height).astype(int)
    y1 = np.clip(np.floor(hi[:, 1]) + 1, 0, cam.height).astype(int)
    x1, y1 = np.maximum(x1, x0), np.maximum(y1, y0)
    n_in = sat[y1, x1] - sat[y0, x1] - sat[y1, x0] + sat[y0, x0]
    cand = (prox.valid | prox.ambiguous).numpy()
    return np.nonzero(cand & (n_in > 0))[0]


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


@pytest.mark.parametrize("basis", ["power", "trigonometric"])
def test_camera_batch_gradients_are_the_sum_over_cameras(basis):
    """Two cameras at 100x75 (a ragged tail in both axes) in one launch: each
    Gaussian's gradient is the sum of its gradients through either image, so
    the batched backward is checked against the sum of the oracle's float64
    autograd per camera (grads.hip accumulates the cameras' entries of a
    Gaussian in one pass). Ambiguous pixels and pixels whose degenerate-measure
    flag differs take no upstream gradient, per camera."""
    scene, _, opts = W.w1_small()
    opts.basis = basis
    cams = [W.camera_on_axis(3.0, 100, 75),
            W.camera_look_at((2.0, 1.0, -2.5), (0, 0, 0), (0, 1, 0), 100, 75)]
    _, saved, _ = gpu_render(scene, cams, opts)
    rng = np.random.default_rng(61)
    g_img = rng.normal(size=(len(cams), 75 * 100, 3))
    ref = {k: 0.0 for k in GROUPS}
    for i, cam in enumerate(cams):
        tol_m, tol_o = tolerances(proxy_error(scene, cam, opts))
        ri = oracle.render_image(scene, cam, opts, margin_tol=tol_m, orient_eps=tol_o)
        skip = ri["ambiguous"] | ((saved[i].reshape(-1, 8)[:, 7] < 0) != ri["fallback"])
        log(f"[grad batch {basis}] camera {i}: pixels without upstream gradient {int(skip.sum())}")
        assert skip.sum() <= 0.01 * len(skip)
        g_img[i][skip] = 0.0
        r = oracle.render_backward(scene, cam, opts, g_img[i])
        for k in GROUPS:
            ref[k] = ref[k] + r[k]
    gpu, _ = _gpu_grads(scene, cams, opts, g_img)
    assert _check(gpu, ref, f"two-camera batch {basis}")
