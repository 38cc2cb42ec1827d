"""Trigonometric moments (Sec. 3.2, Eqs. 13-14, App. C) on the GPU against the
oracle (oracle.trig): the moments of every covering Gaussian on the circle,
the reconstruction on the circle at each quadrature edge, Eq. 7 and Eq. 15.

Forward bar: max-abs image error <= 1e-4 over the pixels the parity
protocol keeps; besides the coverage band it excludes pixels whose
degenerate-measure flag (the Toeplitz matrix mixed with the uniform measure)
differs between the two sides, and pixels where an atom of the
reconstruction lies within oracle.trig.CUT_BAND of the cut at one of the
pixel's queries (its side of the cut, which moves the optical depth by the
atom's weight, is then decided by input rounding), counted and bounded: at
most 1% of W1's pixels and 2% of W2's sample (measured 0.1-0.2% and
0.5-1.0%). Backward bar: that of
the power moments (tests/test_gpu_backward.py), 1e-3 relative per parameter
group and element by element."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_helpers import compare, gpu_render, log, proxy_error, tolerances
from tests.test_gpu_forward import _sample_pixels

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.mark.parametrize("k_mom,n_int", [(4, 3), (4, 5), (6, 3), (6, 5)])
def test_trig_w1_full_image(k_mom, n_int):
    scene, cams, opts = W.w1_small()
    opts.basis = "trigonometric"
    opts.n_moments = k_mom
    opts.n_intervals = n_int
    img, saved, st = gpu_render(scene, cams, opts)
    tol_m, tol_o = tolerances(proxy_error(scene, cams[0], opts))
    ref = oracle.render_image(scene, cams[0], opts, margin_tol=tol_m, orient_eps=tol_o)
    mx, _ = compare(img[0].reshape(-1, 3), ref, f"trig W1 K={k_mom} N={n_int}", max_excluded=0.01,
                    gpu_saved=saved[0].reshape(-1, 8))
    assert mx <= TOL
    m0_err = np.abs(saved[0].reshape(-1, 8)[:, 6] - ref["moments"][:, 0])
    assert m0_err.max() < 1e-4 * max(1.0, ref["moments"][:, 0].max())


@pytest.mark.parametrize("k_mom", [4, 6])
def test_trig_w2_full_size_sampled(k_mom):
    """500k Gaussians at 1920x1080 in the benchmark's launch configuration;
    20,000 sampled pixels."""
    scene, cams, opts = W.w2_clusters(n_moments=k_mom)
    opts.basis = "trigonometric"
    cam = cams[0]
    img, saved, st = gpu_render(scene, cams, opts, on_device=True)
    pix = _sample_pixels(scene, cam, n_random=10_000, n_dense=10_000)
    tol_m, tol_o = tolerances(proxy_error(scene, cam, opts))
    ref = oracle.render_image(scene, cam, opts, pixels=pix, margin_tol=tol_m, orient_eps=tol_o,
                              max_pixels=len(pix))
    log(f"[trig w2 K={k_mom}] sampled={len(pix)} pairs={ref['n_pairs']}")
    mx, _ = compare(img[0].reshape(-1, 3)[pix], ref, f"trig W2 K={k_mom}", max_excluded=0.02,
                    gpu_saved=saved[0].reshape(-1, 8)[pix])
    assert mx <= TOL


def test_trig_single_colour_scene_is_exact():
    """One colour everywhere: Eq. 15 makes the image exact whatever the
    reconstruction (c (1 - e^-m0) + background e^-m0)."""
    scene, cams, opts = W.w1_small()
    opts.basis = "trigonometric"
    scene.colors[:] = np.array([0.3, 0.6, 0.9], np.float32)
    img, saved, st = gpu_render(scene, cams, opts)
    m0 = saved[0].reshape(-1, 8)[:, 6]
    o = saved[0].reshape(-1, 8)[:, 3]
    ok = o >= 1e-6
    expect = np.array([0.3, 0.6, 0.9])[None] * (1 - np.exp(-m0))[:, None]
    assert np.abs(img[0].reshape(-1, 3)[ok] - expect[ok]).max() < 2e-6


def test_trig_ragged_camera_batch_equals_each_camera_alone():
    """Two cameras at 100x75 (a ragged tail in both axes) in one launch, K = 6:
    each batched image equals the camera rendered alone, bit for bit, and the
    oracle within the forward bar."""
    scene, _, opts = W.w1_small()
    opts.basis = "trigonometric"
    opts.n_moments = 6
    cams = [W.camera_on_axis(3.0, 100, 75),
            W.camera_look_at((2.0, 1.0, -2.5), (0, 0, 0), (0, 1, 0), 100, 75)]
    batch, bsaved, _ = gpu_render(scene, cams, opts)
    for i, cam in enumerate(cams):
        single, ssaved, _ = gpu_render(scene, [cam], opts)
        assert np.array_equal(batch[i], single[0])
        assert np.array_equal(bsaved[i], ssaved[0])
        tol_m, tol_o = tolerances(proxy_error(scene, cam, opts))
        ref = oracle.render_image(scene, cam, opts, margin_tol=tol_m, orient_eps=tol_o)
        mx, _ = compare(single[0].reshape(-1, 3), ref, f"trig ragged 100x75 camera {i}", max_excluded=0.01,
                        gpu_saved=ssaved[0].reshape(-1, 8))
        assert mx <= TOL


def _trig_grads(scene, cams, opts, g_img):
    from tests.test_gpu_backward import _gpu_grads
    return _gpu_grads(scene, cams, opts, g_img)


@pytest.mark.parametrize("k_mom,n_int", [(4, 3), (4, 5), (6, 3)])
def test_trig_backward_fd_subset_vs_oracle_autograd(k_mom, n_int):
    """200 Gaussians of one cluster, 64x64, full coverage: the GPU adjoint of
    the reconstruction on the circle (trig_adjoint) and of Eq. 14
    (trig_moment_grads) against float64 autograd of the oracle."""
    from tests.test_gpu_backward import _check
    scene, cams, opts = W.w3_fd_subset()
    scene = scene.subset(np.arange(200))
    opts.basis = "trigonometric"
    opts.n_moments = k_mom
    opts.n_intervals = n_int
    rng = np.random.default_rng(40 + n_int + k_mom)
    g_img = rng.normal(size=(64 * 64, 3))
    gpu, _ = _trig_grads(scene, cams, opts, g_img)
    ref = oracle.render_backward(scene, cams[0], opts, g_img)
    assert _check(gpu, ref, f"trig fd-subset K={k_mom} N={n_int}")


@pytest.mark.parametrize("k_mom", [4, 6])
def test_trig_backward_w1_vs_oracle_autograd(k_mom):
    """The real proxy coverage (W1). Pixels whose coverage decision is
    ambiguous, or whose degenerate-measure flag differs between the two sides,
    take no upstream gradient."""
    from tests.test_gpu_backward import _check
    scene, cams, opts = W.w1_small()
    opts.basis = "trigonometric"
    opts.n_moments = k_mom
    cam = cams[0]
    tol_m, tol_o = tolerances(proxy_error(scene, cam, opts))
    ref_img = oracle.render_image(scene, cam, opts, margin_tol=tol_m, orient_eps=tol_o)
    _, saved, _ = gpu_render(scene, cams, opts)
    flag_gpu = saved[0].reshape(-1, 8)[:, 7] < 0
    skip = ref_img["ambiguous"] | (flag_gpu != ref_img["fallback"])
    log(f"[trig grad W1 K={k_mom}] pixels without upstream gradient: {int(skip.sum())}")
    assert skip.sum() <= 0.01 * len(skip)
    rng = np.random.default_rng(47)
    g_img = rng.normal(size=(cam.width * cam.height, 3))
    g_img[skip] = 0.0
    gpu, _ = _trig_grads(scene, cams, opts, g_img)
    ref = oracle.render_backward(scene, cam, opts, g_img)
    assert _check(gpu, ref, f"trig W1 K={k_mom}")
