"""Seeded synthetic scenes and cameras for moment-based 3D Gaussian splatting.

This module only draws inputs. It holds none of the rendering arithmetic and is
shared by the CPU oracle, the tests and the benchmark, so that every consumer
sees identical float32 arrays for a given workload and seed.

Conventions (the paper leaves them open; see the scene-parameterisation
paragraph of Sec. 3.1, which defers to the original 3DGS parameterisation):

* Gaussian parameters are float32 structure-of-arrays:
  ``means[n,3]``, ``scales[n,3]`` (linear, > 0), ``quats[n,4]`` as (w, x, y, z),
  ``densities[n]`` (the non-negative weight w_i, softplus already applied),
  ``colors[n,3]`` (RGB) or ``colors[n,(d+1)^2,3]`` (SH coefficients, degree d).
* A camera is a world-to-camera rigid transform ``[R | t]`` (row-major 3x4;
  x_cam = R x_world + t) with OpenCV axes (x right, y down, z forward) and
  pinhole intrinsics fx, fy, cx, cy; pixel (x, y) has its centre at
  (x + 0.5, y + 0.5).
* Draw order for a scene: cluster centres, cluster assignments, offsets,
  log-scales, quaternions, densities, colours.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np


@dataclasses.dataclass
class Scene:
    means: np.ndarray
    scales: np.ndarray
    quats: np.ndarray
    densities: np.ndarray
    colors: np.ndarray
    sh_degree: int  # -1: colors are RGB

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Scene":
        return Scene(self.means[idx], self.scales[idx], self.quats[idx],
                     self.densities[idx], self.colors[idx], self.sh_degree)

    def copy(self) -> "Scene":
        return Scene(self.means.copy(), self.scales.copy(), self.quats.copy(),
                     self.densities.copy(), self.colors.copy(), self.sh_degree)


@dataclasses.dataclass
class Camera:
    world_to_cam: np.ndarray  # [3,4] float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    t_near: float = 0.2
    background: tuple = (0.0, 0.0, 0.0)

    def __post_init__(self):
        # the library takes float32 camera parameters: round them here so
        # every consumer sees exactly the values the GPU path receives
        f32 = lambda x: float(np.float32(x))
        self.world_to_cam = np.asarray(self.world_to_cam, np.float32)
        self.fx, self.fy, self.cx, self.cy = f32(self.fx), f32(self.fy), f32(self.cx), f32(self.cy)
        self.t_near = f32(self.t_near)
        self.background = tuple(f32(b) for b in self.background)

    @property
    def origin(self) -> np.ndarray:
        r = self.world_to_cam[:, :3].astype(np.float64)
        t = self.world_to_cam[:, 3].astype(np.float64)
        return -r.T @ t


@dataclasses.dataclass
class Options:
    """Method constants. Defaults are the values the paper prints
    (confidence c, sample-spread kappa, bound interpolation beta) and the
    readings for the ones it leaves open (N intervals, epsilon)."""
    n_moments: int = 4          # K power moments beyond m_0 (K+1 values)
    n_intervals: int = 3        # N quadrature intervals (N+1 edges)
    kappa: float = 3.0          # sample spread, App. B
    conf_c: float = 0.01        # confidence level of the screen proxy, App. D
    beta: float = 0.25          # bound interpolation, Sec. 3.2
    eps: float = 1e-6           # clamp of Eq. 15's denominator
    full_coverage: bool = False  # debug: every Gaussian covers every pixel
    basis: str = "power"        # moment basis: "power" (Eqs. 10-12) or "trigonometric" (Eqs. 13-14)

    def __post_init__(self):
        # the library takes these constants as float32
        for k in ("kappa", "conf_c", "beta", "eps"):
            setattr(self, k, float(np.float32(getattr(self, k))))


def intrinsics_for(width: int, height: int, vfov_deg: float = 60.0):
    """Pinhole intrinsics for a vertical field of view, square pixels,
    principal point at the image centre."""
    f = (height / 2.0) / math.tan(math.radians(vfov_deg) / 2.0)
    return f, f, width / 2.0, height / 2.0


def camera_on_axis(distance: float, width: int, height: int,
                   vfov_deg: float = 60.0, t_near: float = 0.2) -> Camera:
    """Camera at (0, 0, -distance) looking along +z at the origin."""
    w2c = np.zeros((3, 4), np.float32)
    w2c[:, :3] = np.eye(3, dtype=np.float32)
    w2c[2, 3] = distance
    fx, fy, cx, cy = intrinsics_for(width, height, vfov_deg)
    return Camera(w2c, fx, fy, cx, cy, width, height, t_near)


def camera_look_at(position, target, up, width: int, height: int,
                   vfov_deg: float = 60.0, t_near: float = 0.2) -> Camera:
    """OpenCV-axis camera at ``position`` looking at ``target``."""
    c = np.asarray(position, np.float64)
    fwd = np.asarray(target, np.float64) - c
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, np.float64))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    r = np.stack([right, down, fwd])
    w2c = np.zeros((3, 4), np.float64)
    w2c[:, :3] = r
    w2c[:, 3] = -r @ c
    fx, fy, cx, cy = intrinsics_for(width, height, vfov_deg)
    return Camera(w2c.astype(np.float32), fx, fy, cx, cy, width, height, t_near)


def random_cameras(n: int, radius: float, width: int, height: int, seed: int,
                   vfov_deg: float = 60.0) -> List[Camera]:
    """Cameras on a sphere of ``radius`` (directions uniform on S^2) looking at
    the origin with world up +y."""
    rng = np.random.default_rng(seed)
    cams = []
    while len(cams) < n:
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        if abs(v[1]) > 0.995:  # look direction (anti)parallel to up
            continue
        cams.append(camera_look_at(radius * v, (0, 0, 0), (0, 1, 0),
                                   width, height, vfov_deg))
    return cams


def _unit_quats(rng, n):
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def uniform_scene(n: int, seed: int, extent: float = 1.0,
                  log_scale_mean: float = -3.0, log_scale_std: float = 0.5,
                  density_sigma: float = 1.0) -> Scene:
    """Means uniform in [-extent, extent]^3, per-axis log-scales normal,
    random unit quaternions, log-normal densities, RGB uniform in [0, 1]."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-extent, extent, size=(n, 3))
    log_s = rng.normal(log_scale_mean, log_scale_std, size=(n, 3))
    quats = _unit_quats(rng, n)
    dens = rng.lognormal(0.0, density_sigma, size=n)
    rgb = rng.uniform(0.0, 1.0, size=(n, 3))
    return Scene(means.astype(np.float32), np.exp(log_s).astype(np.float32),
                 quats.astype(np.float32), dens.astype(np.float32),
                 rgb.astype(np.float32), -1)


def clustered_scene(n: int, seed: int, n_clusters: int = 64,
                    centre_extent: float = 4.0, offset_std: float = 0.3,
                    log_scale_mean: float = -4.0, log_scale_std: float = 0.7,
                    density_sigma: float = 1.5, sh_degree: int = 3,
                    sh_std: float = 0.2, centres: Optional[np.ndarray] = None
                    ) -> Scene:
    """Gaussians drawn from isotropic clusters: centres uniform in
    [-centre_extent, centre_extent]^3, members offset by N(0, offset_std^2 I),
    per-axis log-scales normal, log-normal densities, SH coefficients normal."""
    rng = np.random.default_rng(seed)
    if centres is None:
        centres = rng.uniform(-centre_extent, centre_extent, size=(n_clusters, 3))
    else:
        centres = np.asarray(centres, np.float64).reshape(-1, 3)
        n_clusters = centres.shape[0]
    assign = rng.integers(0, n_clusters, size=n)
    offsets = rng.normal(0.0, offset_std, size=(n, 3))
    means = centres[assign] + offsets
    log_s = rng.normal(log_scale_mean, log_scale_std, size=(n, 3))
    quats = _unit_quats(rng, n)
    dens = rng.lognormal(0.0, density_sigma, size=n)
    if sh_degree < 0:
        colors = rng.uniform(0.0, 1.0, size=(n, 3))
    else:
        colors = rng.normal(0.0, sh_std, size=(n, (sh_degree + 1) ** 2, 3))
    return Scene(means.astype(np.float32), np.exp(log_s).astype(np.float32),
                 quats.astype(np.float32), dens.astype(np.float32),
                 colors.astype(np.float32), sh_degree)


# ---------------------------------------------------------------------------
# Named workloads.
# ---------------------------------------------------------------------------

def w1_small(seed: int = 0):
    """2,000 Gaussians, means U[-1,1]^3, log-scales N(-3,0.5), densities
    LogNormal(0,1), RGB; 128x128 camera at distance 3, 60 deg fov, K=4, N=3."""
    scene = uniform_scene(2000, seed)
    cam = camera_on_axis(3.0, 128, 128)
    return scene, [cam], Options(n_moments=4)


def w2_clusters(n: int = 500_000, seed: int = 1, n_moments: int = 4,
                width: int = 1920, height: int = 1080, distance: float = 10.0):
    """500k Gaussians in 64 isotropic clusters, SH degree 3, 1080p camera."""
    scene = clustered_scene(n, seed)
    cam = camera_on_axis(distance, width, height)
    return scene, [cam], Options(n_moments=n_moments)


def w3_train(n: int = 1_000_000, seed: int = 2, width: int = 1600, height: int = 1064,
             distance: float = 10.0, perturb_std: float = 0.01):
    """Training step: the W2 generator at 1M Gaussians, 1600x1064; the target
    scene is a copy with means perturbed by N(0, perturb_std^2)."""
    scene = clustered_scene(n, seed)
    rng = np.random.default_rng(seed + 1000)
    target = scene.copy()
    target.means = (target.means.astype(np.float64)
                    + rng.normal(0.0, perturb_std, size=target.means.shape)).astype(np.float32)
    cam = camera_on_axis(distance, width, height)
    return scene, target, [cam], Options(n_moments=4)


def w3_fd_subset(seed: int = 2):
    """500 Gaussians of one cluster at the origin, 64x64 camera at distance 2,
    full coverage (smooth in every parameter) for finite differences."""
    scene = clustered_scene(500, seed, centres=np.zeros((1, 3)))
    cam = camera_on_axis(2.0, 64, 64)
    return scene, [cam], Options(n_moments=4, full_coverage=True)


def w4_surrogate(n: int = 500_000, seed: int = 3, n_train_cams: int = 32,
                 n_eval_cams: int = 8, width: int = 1920, height: int = 1080):
    """The W2 scene with K=6, 32 training cameras and 8 held-out cameras at
    radius 10 looking at the origin."""
    scene = clustered_scene(n, seed)
    train = random_cameras(n_train_cams, 10.0, width, height, seed)
    held = random_cameras(n_eval_cams, 10.0, width, height, seed + 1)
    return scene, train, held, Options(n_moments=6)


def w5_large(n: int = 3_000_000, seed: int = 5, n_cams: int = 8,
             width: int = 3840, height: int = 2160):
    """3M Gaussians in 256 clusters, 8 cameras at 3840x2160."""
    scene = clustered_scene(n, seed, n_clusters=256)
    cams = random_cameras(n_cams, 10.0, width, height, seed)
    return scene, cams, Options(n_moments=4)
