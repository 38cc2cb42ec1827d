"""The seeded input generators against each workload's stated recipe (the
docstrings of workloads/__init__.py): sizes, value distributions, camera
placement and determinism.
Statistical checks use tolerances several standard errors wide (the draws
are seeded, so each check is deterministic)."""
import math

import numpy as np
import pytest

import workloads as W


def _project(cam, x):
    xc = cam.world_to_cam[:, :3].astype(np.float64) @ np.asarray(x, np.float64) + cam.world_to_cam[:, 3]
    return np.array([cam.fx * xc[0] / xc[2] + cam.cx, cam.fy * xc[1] / xc[2] + cam.cy]), xc[2]


def _check_common(scene):
    q = scene.quats.astype(np.float64)
    assert np.allclose(np.linalg.norm(q, axis=1), 1.0, atol=1e-6)
    assert np.all(scene.scales > 0) and np.all(scene.densities > 0)
    for a in (scene.means, scene.scales, scene.quats, scene.densities, scene.colors):
        assert a.dtype == np.float32 and np.all(np.isfinite(a))


def test_small_scene_recipe():
    scene, cams, opts = W.w1_small()
    assert scene.n == 2000 and scene.sh_degree == -1 and scene.colors.shape == (2000, 3)
    _check_common(scene)
    assert scene.means.min() >= -1.0 and scene.means.max() <= 1.0
    ls = np.log(scene.scales.astype(np.float64))
    assert abs(ls.mean() + 3.0) < 0.03 and abs(ls.std() - 0.5) < 0.02
    ld = np.log(scene.densities.astype(np.float64))
    assert abs(ld.mean()) < 0.07 and abs(ld.std() - 1.0) < 0.04
    assert scene.colors.min() >= 0.0 and scene.colors.max() <= 1.0
    (cam,) = cams
    assert (cam.width, cam.height) == (128, 128)
    assert np.allclose(cam.origin, [0.0, 0.0, -3.0], atol=1e-6)
    # 60 degree vertical field of view, principal point at the centre
    assert math.isclose(cam.fy, 64.0 / math.tan(math.radians(30.0)), rel_tol=1e-6)
    assert (cam.cx, cam.cy) == (64.0, 64.0)
    assert (opts.n_moments, opts.n_intervals, opts.basis) == (4, 3, "power")
    assert (opts.kappa, opts.beta) == (3.0, 0.25) and math.isclose(opts.conf_c, 0.01, rel_tol=1e-6)


def test_clustered_scene_recipe():
    # the 500k-Gaussian 1080p generator, at a tenth of the size
    scene = W.clustered_scene(50_000, 1)
    assert scene.sh_degree == 3 and scene.colors.shape == (50_000, 16, 3)
    _check_common(scene)
    ls = np.log(scene.scales.astype(np.float64))
    assert abs(ls.mean() + 4.0) < 0.01 and abs(ls.std() - 0.7) < 0.01
    ld = np.log(scene.densities.astype(np.float64))
    assert abs(ld.mean()) < 0.03 and abs(ld.std() - 1.5) < 0.02
    assert abs(scene.colors.astype(np.float64).std() - 0.2) < 0.002
    # 64 clusters with centres in [-4, 4]^3 and N(0, 0.3^2) offsets: every
    # mean lies within 6 offset deviations of the cube, and the means group
    # around 64 centres (re-drawn from the same seed)
    assert np.abs(scene.means).max() <= 4.0 + 6 * 0.3
    rng = np.random.default_rng(1)
    centres = rng.uniform(-4.0, 4.0, size=(64, 3))
    d = np.linalg.norm(scene.means[:, None, :].astype(np.float64) - centres[None], axis=2).min(axis=1)
    # the distance to the nearest centre is at most that to the own centre,
    # a chi distribution with 3 degrees of freedom scaled by 0.3
    assert np.quantile(d, 0.99) < 0.3 * 3.4


def test_full_size_frame_camera_and_options():
    cam = W.camera_on_axis(10.0, 1920, 1080)
    assert np.allclose(cam.origin, [0.0, 0.0, -10.0], atol=1e-5)
    uv, depth = _project(cam, [0.0, 0.0, 0.0])
    assert np.allclose(uv, [960.0, 540.0]) and math.isclose(depth, 10.0, rel_tol=1e-6)
    for k in (4, 6, 8):
        assert W.Options(n_moments=k).n_moments == k


def test_training_target_is_the_scene_with_perturbed_means():
    # the training-step generator (1M Gaussians at 1600x1064), at 20k Gaussians
    scene, target, cams, opts = W.w3_train(n=20_000)
    d = (target.means - scene.means).astype(np.float64)
    assert abs(d.std() - 0.01) < 2e-4 and abs(d.mean()) < 2e-4
    for k in ("scales", "quats", "densities", "colors"):
        assert np.array_equal(getattr(target, k), getattr(scene, k))
    assert (cams[0].width, cams[0].height) == (1600, 1064)


def test_cameras_on_a_sphere_look_at_the_origin():
    cams = W.random_cameras(8, 10.0, 3840, 2160, 5)
    assert len(cams) == 8
    for cam in cams:
        assert (cam.width, cam.height) == (3840, 2160)
        assert math.isclose(np.linalg.norm(cam.origin), 10.0, rel_tol=1e-5)
        r = cam.world_to_cam[:, :3].astype(np.float64)
        assert np.allclose(r @ r.T, np.eye(3), atol=1e-6) and np.linalg.det(r) > 0
        uv, depth = _project(cam, [0.0, 0.0, 0.0])
        assert np.allclose(uv, [1920.0, 1080.0], atol=1e-2) and math.isclose(depth, 10.0, rel_tol=1e-5)
    # held-out cameras come from another seed
    train = W.random_cameras(4, 10.0, 64, 64, 3)
    held = W.random_cameras(4, 10.0, 64, 64, 4)
    assert not any(np.allclose(a.origin, b.origin) for a in train for b in held)


@pytest.mark.parametrize("gen", [lambda s: W.uniform_scene(500, s), lambda s: W.clustered_scene(500, s)])
def test_generators_are_deterministic_per_seed(gen):
    a, b, c = gen(7), gen(7), gen(8)
    for k in ("means", "scales", "quats", "densities", "colors"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
        assert not np.array_equal(getattr(a, k), getattr(c, k))
