"""The tabulated schedule on the GPU (mb_render_forward_tabulated) against the
oracle's schedule (oracle.surrogate.tabulated): per pixel, the reconstruction
at 32 nodes of the standardised query on [-4, 4], interpolated linearly at
every quadrature edge, with the moment bounds of Sec. 3.2 or the learned
surrogate at the nodes.

Bars. Bounds: max-abs image error <= 1e-4 over the pixels the parity protocol
keeps (as for the per-query render; excluded pixels counted and bounded).
Surrogate: the statistical bar of the per-query surrogate render (its inputs
and hidden activations are rounded to bf16 on both sides, and float32 against
float64 inputs can round to neighbouring bf16 values at ties)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from oracle import surrogate as S
from tests.gpu_helpers import compare, log, proxy_error, tolerances
from tests.test_gpu_forward import _sample_pixels

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _tab_render(scene, cams, opts, packed=None, n_nodes=32):
    import paper_2512_11800_amd as M
    g = M.Gaussians.from_scene(scene)
    img, saved, _ = M.render_forward_tabulated(g, cams, opts, packed, n_nodes=n_nodes)
    torch.cuda.synchronize()
    return img.cpu().numpy().astype(np.float64), saved.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("k_mom,n_int", [(4, 3), (6, 3), (4, 5), (6, 5)])
def test_tabulated_bounds_w1(k_mom, n_int):
    import paper_2512_11800_amd as M
    scene, cams, opts = W.w1_small()
    opts.n_moments = k_mom
    opts.n_intervals = n_int
    img, saved = _tab_render(scene, cams, opts)
    tol_m, tol_o = tolerances(proxy_error(scene, cams[0], opts))
    model = S.tabulated(S.bounds_model(k_mom // 2, opts.beta))
    ref = oracle.render_image(scene, cams[0], opts, margin_tol=tol_m, orient_eps=tol_o, tau_model=model)
    mx, _ = compare(img[0].reshape(-1, 3), ref, f"tabulated bounds W1 K={k_mom} N={n_int}",
                    max_excluded=0.01, gpu_saved=saved[0].reshape(-1, 8))
    assert mx <= TOL
    # against the per-query render: the schedule's own error, logged
    plain, _, _ = M.render_forward(M.Gaussians.from_scene(scene), cams, opts)
    d = np.abs(plain[0].cpu().numpy().reshape(-1, 3) - img[0].reshape(-1, 3))
    log(f"[tabulated K={k_mom} N={n_int}] |tabulated - per-query| max={d.max():.3e} mean={d.mean():.3e}")


def test_tabulated_bounds_w2_full_size_sampled():
    """500k Gaussians at 1920x1080; 5,000 sampled pixels."""
    scene, cams, opts = W.w2_clusters(n_moments=4)
    cam = cams[0]
    img, saved = _tab_render(scene, cams, opts)
    pix = _sample_pixels(scene, cam, n_random=2_500, n_dense=2_500)
    tol_m, tol_o = tolerances(proxy_error(scene, cam, opts))
    ref = oracle.render_image(scene, cam, opts, pixels=pix, margin_tol=tol_m, orient_eps=tol_o,
                              max_pixels=len(pix), tau_model=S.tabulated(S.bounds_model(2, opts.beta)))
    mx, _ = compare(img[0].reshape(-1, 3)[pix], ref, "tabulated bounds W2", max_excluded=0.01,
                    gpu_saved=saved[0].reshape(-1, 8)[pix])
    assert mx <= TOL


@pytest.mark.parametrize("n_int", [3, 5])
def test_tabulated_surrogate_w1(n_int):
    from paper_2512_11800_amd import surrogate as G
    scene, cams, opts = W.w1_small()
    opts.n_moments = 6
    opts.n_intervals = n_int
    cam = cams[0]
    theta = S.init_params(21)
    packed = G.mlp_pack(torch.tensor(theta, dtype=torch.float32, device="cuda"))
    img, _ = _tab_render(scene, cams, opts, packed)
    img = img[0].reshape(-1, 3)
    tol_m, tol_o = tolerances(proxy_error(scene, cam, opts))
    theta32 = theta.astype(np.float32).astype(np.float64)
    ref = oracle.render_image(scene, cam, opts, margin_tol=tol_m, orient_eps=tol_o,
                              tau_model=S.tabulated(S.tau_model(theta32)))
    keep = ~ref["ambiguous"]
    e = np.abs(img - ref["image"]).max(-1)[keep]
    q999 = float(np.quantile(e, 0.999))
    log(f"[tabulated surrogate N={n_int}] pixels {keep.sum()} median={np.median(e):.2e} "
        f"p99.9={q999:.2e} max={e.max():.2e}")
    assert np.all(np.isfinite(img))
    assert np.median(e) < 1e-6 and q999 < 1e-4 and e.max() < 2e-3


def test_tabulated_node_counts_and_errors():
    """More nodes move the tabulated render toward the per-query render;
    node counts outside [2, 256] and the trigonometric basis are refused."""
    import paper_2512_11800_amd as M
    scene, cams, opts = W.w1_small()
    g = M.Gaussians.from_scene(scene)
    plain, _, _ = M.render_forward(g, cams, opts)
    plain = plain.cpu().numpy()
    errs = []
    for n in (8, 32, 128):
        img, _, _ = M.render_forward_tabulated(g, cams, opts, None, n_nodes=n)
        errs.append(float(np.abs(img.cpu().numpy() - plain).mean()))
    log(f"[tabulated] mean |tabulated - per-query| for 8/32/128 nodes: {errs}")
    assert errs[2] < errs[1] < errs[0]
    for bad in (1, 257):
        with pytest.raises(M.MbError, match="n_nodes"):
            M.render_forward_tabulated(g, cams, opts, None, n_nodes=bad)
    opts.basis = "trigonometric"
    with pytest.raises(M.MbError, match="power moments"):
        M.render_forward_tabulated(g, cams, opts, None)
