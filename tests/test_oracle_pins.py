"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test ties one part of the oracle to something other than itself:
closed forms, numeric integration, textbook cases, linear programming,
library special functions, invariants, limits and finite differences.
"""
import dataclasses
import math
import warnings

import numpy as np
import pytest
import torch
from scipy import integrate
from scipy.optimize import linprog
from scipy.special import erfc, sph_harm_y

import oracle
import workloads as W
from oracle.bounds import bound_tau, canonical_representation
from oracle.geometry import quat_to_rot, ray_gaussian, real_sh_basis
from oracle.moments import linearised_warp, particle_moments, power_transform, warp, warp_prime
from oracle.proxy import screen_proxy
from oracle.quadrature import normal_quantiles, particle_quadrature
from oracle.render import render_pixels, scene_tensors

DT = torch.float64


def _t(x):
    return torch.as_tensor(np.asarray(x, np.float64))


# ---------------------------------------------------------------------------
# Eqs. 4-6: the ray-space 1D Gaussian equals the 3D density along the ray.
# ---------------------------------------------------------------------------

def test_ray_gaussian_matches_3d_density():
    rng = np.random.default_rng(11)
    for _ in range(20):
        mean = rng.normal(size=3) * 2
        scale = np.exp(rng.normal(-1, 0.5, 3))
        q = rng.normal(size=4)
        w = rng.lognormal()
        o = rng.normal(size=3) * 3
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        r = quat_to_rot(_t(q)).numpy()
        prec = r @ np.diag(1 / scale ** 2) @ r.T
        mu, sig, om = ray_gaussian(_t(o), _t(d), _t(mean), _t(r), _t(scale), _t(w))
        for t in rng.uniform(-5, 5, 7):
            x = o + t * d - mean
            ref = w * math.exp(-0.5 * x @ prec @ x)
            got = om.item() * math.exp(-(t - mu.item()) ** 2 / (2 * sig.item() ** 2))
            assert got == pytest.approx(ref, rel=1e-9, abs=1e-300)


def test_quaternion_rotation_is_orthonormal_and_matches_axis_angle():
    ang = 0.7
    axis = np.array([1.0, 2.0, -0.5])
    axis /= np.linalg.norm(axis)
    q = np.concatenate([[math.cos(ang / 2)], math.sin(ang / 2) * axis]) * 3.0  # unnormalised
    r = quat_to_rot(_t(q)).numpy()
    k = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    rodrigues = np.eye(3) + math.sin(ang) * k + (1 - math.cos(ang)) * k @ k
    assert np.abs(r - rodrigues).max() < 1e-14
    assert np.abs(r @ r.T - np.eye(3)).max() < 1e-14


# ---------------------------------------------------------------------------
# Warp (Sec. 3.2): Barron's power transform and its normalisation.
# ---------------------------------------------------------------------------

def test_power_transform_special_cases():
    x = np.linspace(0, 10, 51)
    assert np.allclose(power_transform(x, 1.0 + 1e-12), x, atol=1e-9)        # identity
    assert np.allclose(power_transform(x, 2.0), x + x * x / 2)                 # quadratic
    assert np.allclose(power_transform(x, 1e-9), np.log1p(x), atol=1e-7)      # log limit
    assert np.allclose(power_transform(x, -1.5), 5 / 3 * (1 - (1 + x / 2.5) ** -1.5))
    h = 1e-6
    for lam in (-1.5, 0.5, 2.0):
        slope = (power_transform(h, lam) - power_transform(-h, lam)) / (2 * h)
        assert slope == pytest.approx(1.0, abs=1e-8)


def test_warp_maps_near_to_zero_far_to_one_and_derivative():
    tn = 0.2
    assert warp(tn, tn) == pytest.approx(0.0, abs=1e-15)
    assert warp(1e12, tn) == pytest.approx(1.0, abs=1e-12)
    t = np.linspace(0.2, 30, 40)
    h = 1e-5
    fd = (warp(t + h, tn) - warp(t - h, tn)) / (2 * h)
    assert np.allclose(warp_prime(t, tn), fd, rtol=1e-8)
    assert np.all(np.diff(warp(t, tn)) > 0)


# ---------------------------------------------------------------------------
# Eqs. 10-12: the recurrence equals direct numerical integration of the
# linearised warp powers against the ray density on [t_n, inf); m_0 equals
# the exact optical depth of the particle (no approximation).
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mu,sig,om", [(5.0, 0.3, 2.0), (0.5, 0.4, 1.0), (0.1, 0.2, 3.0),
                                       (12.0, 0.02, 5.0), (-0.5, 0.3, 1.5)])
def test_moment_recurrence_vs_quadrature(mu, sig, om):
    tn, c, s = 0.2, 0.9, 0.01
    m = particle_moments(_t([mu]), _t([sig]), _t([om]), tn, 6, _t([c]), _t([s]))[0].numpy()
    g, gp = (v.item() for v in linearised_warp(_t([mu]), tn, _t([c]), _t([s])))
    for k in range(7):
        f = lambda t: (g + gp * (t - mu)) ** k * om * math.exp(-(t - mu) ** 2 / (2 * sig * sig))
        ref, _ = integrate.quad(f, tn, max(tn, mu) + 40 * sig, limit=400, epsabs=0,
                                epsrel=1e-13, points=[max(tn, mu)])
        assert m[k] == pytest.approx(ref, rel=1e-11, abs=1e-300)


def test_zeroth_moment_is_exact_optical_depth():
    """m_0 of a particle equals int_{t_n}^inf sigma_i(t) dt (Eq. 10)."""
    tn = 0.2
    for mu, sig, om in [(3.0, 0.5, 1.0), (0.3, 0.2, 2.0), (-1.0, 0.7, 0.5)]:
        m0 = particle_moments(_t([mu]), _t([sig]), _t([om]), tn, 0, _t([0.0]), _t([1.0]))[0, 0].item()
        ref, _ = integrate.quad(lambda t: om * math.exp(-(t - mu) ** 2 / (2 * sig * sig)),
                                tn, np.inf, epsabs=0, epsrel=1e-13)
        assert m0 == pytest.approx(ref, rel=1e-12)


def test_raw_moment_lower_bound_constant():
    """App. C: (m_k)_i >= c0 omega mu^k Sigma with c0 = sqrt(pi/2) erf(1) ~ 1.0562,
    checked on raw (unwarped) moments by integration."""
    c0 = math.sqrt(math.pi / 2) * math.erf(1.0)
    assert c0 == pytest.approx(1.0562, abs=1e-4)
    for mu, sig, om, k in [(2.0, 0.3, 1.0, 3), (5.0, 1.0, 0.5, 4)]:
        mk, _ = integrate.quad(lambda t: t ** k * om * math.exp(-(t - mu) ** 2 / (2 * sig * sig)),
                               0.0, np.inf)
        assert mk >= c0 * om * mu ** k * sig


def test_moments_affine_variable_change():
    """Moments in y = (g - c)/s are the binomial transform of moments in g."""
    tn = 0.2
    mu, sig, om = _t([4.0]), _t([0.3]), _t([2.0])
    raw = particle_moments(mu, sig, om, tn, 6, _t([0.0]), _t([1.0]))[0].numpy()
    c, s = 0.93, 0.02
    aff = particle_moments(mu, sig, om, tn, 6, _t([c]), _t([s]))[0].numpy()
    for k in range(7):
        ref = sum(math.comb(k, j) * raw[j] * (-c) ** (k - j) for j in range(k + 1)) / s ** k
        assert aff[k] == pytest.approx(ref, rel=1e-6, abs=1e-9 * abs(raw[0]) / s ** k)


# ---------------------------------------------------------------------------
# Sec. 3.2 reconstruction: canonical representation and bounds.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [2, 3, 4])
def test_canonical_representation_recovers_atomic_measure(n):
    """A measure with n+1 atoms queried at one of its atoms is its own
    canonical representation (uniqueness), so L and U are its step values."""
    rng = np.random.default_rng(n)
    x = np.sort(rng.uniform(-1.5, 1.5, n + 1))
    w = rng.uniform(0.1, 1, n + 1)
    w /= w.sum()
    b = _t([(w * x ** k).sum() for k in range(2 * n + 1)])
    for j in range(n + 1):
        xs, ws = canonical_representation(b[None], _t([x[j]]), n)
        order = np.argsort(xs[0].numpy())
        assert np.abs(xs[0].numpy()[order] - x).max() < 1e-9
        assert np.abs(ws[0].numpy()[order] - w).max() < 1e-9
        m0 = 2.5
        tau, lo, up = bound_tau(m0 * b[None], _t([x[j]]), n, 0.25)
        assert lo.item() == pytest.approx(w[:j].sum(), abs=1e-9)
        assert up.item() == pytest.approx(w[:j + 1].sum(), abs=1e-9)
        assert tau.item() == pytest.approx(m0 * (w[:j].sum() + 0.25 * w[j]), abs=1e-9)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_bounds_are_sharp_lp_bounds(n):
    """L and U are the smallest and largest mass on (-inf, eta) resp.
    (-inf, eta] over all measures with the given moments; compare with a
    linear program over a fine support grid, and bracket the true CDF."""
    grid = np.linspace(-4, 4, 1601)
    dens = np.exp(-(grid + 1) ** 2 / 0.1) + 0.5 * np.exp(-(grid - 1.2) ** 2 / 0.3)
    dens /= dens.sum()
    b = _t([(dens * grid ** k).sum() for k in range(2 * n + 1)])
    a_eq = np.stack([grid ** k for k in range(2 * n + 1)])
    for eta in (-1.5, -0.3, 0.7, 1.9):
        _, lo, up = bound_tau(b[None], _t([eta]), n, 0.25)
        below = (grid < eta).astype(float)
        at = (grid <= eta).astype(float)
        lp_lo = linprog(below, A_eq=a_eq, b_eq=b.numpy(), bounds=(0, None), method="highs").fun
        lp_hi = -linprog(-at, A_eq=a_eq, b_eq=b.numpy(), bounds=(0, None), method="highs").fun
        assert lo.item() == pytest.approx(lp_lo, abs=3e-3)
        assert up.item() == pytest.approx(lp_hi, abs=3e-3)
        true_cdf = (dens * below).sum()
        assert lo.item() <= true_cdf + 1e-12 <= up.item() + 2e-12


@pytest.mark.parametrize("n", [2, 3, 4])
def test_canonical_nodes_reproduce_all_moments_and_christoffel_weight(n):
    rng = np.random.default_rng(7 + n)
    comps = rng.uniform(-1, 1, 5)
    grid = np.linspace(-3, 3, 3001)
    dens = sum(np.exp(-(grid - c) ** 2 / 0.05) for c in comps)
    dens /= dens.sum()
    b = _t([(dens * grid ** k).sum() for k in range(2 * n + 1)])
    h = b[torch.arange(n + 1)[:, None] + torch.arange(n + 1)[None, :]].numpy()
    for eta in np.linspace(-1.5, 1.5, 9):
        xs, ws = canonical_representation(b[None], _t([eta]), n)
        xs, ws = xs[0].numpy(), ws[0].numpy()
        for k in range(2 * n + 1):
            assert (ws * xs ** k).sum() == pytest.approx(b[k].item(), abs=1e-9)
        v = eta ** np.arange(n + 1)
        assert ws[0] == pytest.approx(1.0 / (v @ np.linalg.solve(h, v)), rel=1e-8)
        assert np.all(ws > 0)


def test_tau_monotone_and_bounded():
    rng = np.random.default_rng(3)
    for n in (2, 3, 4):
        for _ in range(5):
            grid = np.linspace(-3, 3, 2001)
            dens = sum(rng.uniform(0.1, 1) * np.exp(-(grid - rng.uniform(-2, 2)) ** 2
                                                     / rng.uniform(0.01, 0.5)) for _ in range(4))
            m = _t([(dens * grid ** k).sum() for k in range(2 * n + 1)]) * 0.01
            etas = _t(np.linspace(-4, 4, 200))
            tau, _, _ = bound_tau(m[None].expand(200, -1), etas, n, 0.25)
            tau = tau.numpy()
            assert np.all(np.diff(tau) >= -1e-10)
            assert tau.min() >= -1e-12 and tau.max() <= m[0].item() * (1 + 1e-12)


def _atoms(n, seed):
    rng = np.random.default_rng(seed)
    x = np.sort(rng.uniform(-1.5, 1.5, n))
    while np.diff(x).min() < 0.3:
        x = np.sort(rng.uniform(-1.5, 1.5, n))
    w = rng.uniform(0.2, 1, n)
    return x, w / w.sum()


@pytest.mark.parametrize("n", [2, 3, 4])
def test_degenerate_measure_is_mixed_with_its_normal(n):
    """Reading for degenerate measures (oracle.bounds.degenerate_mixture): an
    n-atom measure has a singular (n+1)x(n+1) Hankel matrix, so it is flagged
    and replaced by (1 - eps) mu + eps N(mean, var). The mixture's moments
    match numerical integration of that mixture; its bounds bracket the
    mixture's own distribution function (Sec. 3.2: the bounds hold for every
    measure with these moments), are O(eps) apart away from the atoms, and
    are within O(eps) of the atoms' step function."""
    from oracle.bounds import MIX_EPS, degenerate_mixture
    from scipy.stats import norm
    x, w = _atoms(n, 40 + n)
    b = np.array([(w * x ** k).sum() for k in range(2 * n + 1)])
    bu, eps = degenerate_mixture(_t(b)[None], n)
    assert eps.item() == MIX_EPS[0]
    e = eps.item()
    mean, sd = b[1], math.sqrt(b[2] - b[1] ** 2)
    for k in range(2 * n + 1):
        nk = integrate.quad(lambda y: y ** k * norm.pdf(y, mean, sd), -np.inf, np.inf,
                            epsabs=1e-13, epsrel=1e-12)[0]
        assert bu[0, k].item() == pytest.approx((1 - e) * b[k] + e * nk, rel=1e-10, abs=1e-12)
    etas = np.concatenate([(x[:-1] + x[1:]) / 2, [x[0] - 0.4, x[-1] + 0.4]])
    m0 = 1.7
    tau, lo, up = bound_tau(_t(m0 * b)[None].expand(len(etas), -1), _t(etas), n, 0.25)
    lo, up = lo.numpy(), up.numpy()
    step = np.array([w[x < eta].sum() for eta in etas])
    f_mix = (1 - e) * step + e * norm.cdf(etas, mean, sd)
    assert np.all(lo <= f_mix + 1e-12) and np.all(f_mix <= up + 1e-12)
    # U - L is the Christoffel function at eta, the least integral of p^2 over
    # polynomials of degree n with p(eta) = 1; p = prod (y - x_i) / prod (eta - x_i)
    # vanishes on the atoms, so U - L <= eps E_N[p^2]
    for i, eta in enumerate(etas):
        p2 = integrate.quad(lambda y: np.prod((y - x) / (eta - x)) ** 2 * norm.pdf(y, mean, sd),
                            -np.inf, np.inf, epsabs=1e-14, epsrel=1e-10)[0]
        assert up[i] - lo[i] <= e * p2 * (1 + 1e-9)
        assert abs(lo[i] - step[i]) <= e * p2 + e


def test_measures_of_gaussian_sums_are_not_degenerate():
    """The rule leaves the bounds of sums of moderately wide Gaussians alone."""
    from oracle.bounds import degenerate_mixture
    rng = np.random.default_rng(17)
    grid = np.linspace(-4, 4, 4001)
    for n in (2, 3, 4):
        for _ in range(5):
            dens = sum(rng.uniform(0.1, 1) * np.exp(-(grid - rng.uniform(-2, 2)) ** 2
                                                     / rng.uniform(0.1, 0.5)) for _ in range(4))
            b = np.array([(dens * grid ** k).sum() for k in range(2 * n + 1)])
            _, eps = degenerate_mixture(_t(b / b[0])[None], n)
            assert eps.item() == 0.0


def test_degenerate_rule_is_invariant_under_affine_moment_variable():
    """The decision and the mixture commute with an increasing affine map of
    the moment variable, so the bounds do not depend on the pixel's basis."""
    n = 3
    x, w = _atoms(n, 7)
    a_, c_ = 2.7, -0.8
    b = np.array([(w * x ** k).sum() for k in range(2 * n + 1)])
    b2 = np.array([(w * (a_ * x + c_) ** k).sum() for k in range(2 * n + 1)])
    etas = np.array([-1.2, 0.1, 0.9, 1.4])
    t1, _, _ = bound_tau(_t(b)[None].expand(4, -1), _t(etas), n, 0.25)
    t2, _, _ = bound_tau(_t(b2)[None].expand(4, -1), _t(a_ * etas + c_), n, 0.25)
    assert np.abs(t1.numpy() - t2.numpy()).max() < 1e-9


def test_gradient_through_the_degenerate_mixture_vs_central_differences():
    n = 3
    x, w = _atoms(n, 9)
    m = _t(1.3 * np.array([(w * x ** k).sum() for k in range(2 * n + 1)]))
    etas = _t([-0.7, 0.2, 1.1])
    mt = m.clone().requires_grad_(True)
    tau, _, _ = bound_tau(mt[None].expand(3, -1), etas, n, 0.25)
    gw = _t([0.3, -1.1, 0.7])
    (g,) = torch.autograd.grad((tau * gw).sum(), mt)
    # the near-atomic measure is sharply curved: central differences converge
    # as h^2 (4e-5, 4e-7, 1e-8 relative at h = 1e-6, 1e-7, 1e-8)
    h = 1e-8
    fd = []
    for k in range(2 * n + 1):
        mp, mm = m.clone(), m.clone()
        mp[k] += h
        mm[k] -= h
        fp = (bound_tau(mp[None].expand(3, -1), etas, n, 0.25)[0] * gw).sum().item()
        fm = (bound_tau(mm[None].expand(3, -1), etas, n, 0.25)[0] * gw).sum().item()
        fd.append((fp - fm) / (2 * h))
    assert np.abs(np.array(fd) - g.numpy()).max() <= 1e-6 * np.abs(g.numpy()).max()


# ---------------------------------------------------------------------------
# App. B quadrature.
# ---------------------------------------------------------------------------

def test_normal_quantiles_invert_the_normal_cdf():
    for n in (3, 5):
        x = normal_quantiles(n).numpy()
        u = 0.5 * erfc(-x / math.sqrt(2))
        assert np.allclose(u, (np.arange(1, n + 2) - 0.5) / (n + 1), atol=1e-15)
    assert normal_quantiles(3).numpy()[-1] == pytest.approx(1.1503493803760079, abs=1e-12)


def test_quadrature_equals_eq7_literal_form():
    """T_j Delta_j phi(Delta tau_j) sigma_i(t_j) == (T_j - T_{j+1}) sigma_i / sigma_bar_j."""
    mu, sig, om = _t([3.0, 1.0]), _t([0.4, 0.3]), _t([1.5, 0.7])
    tau_fn = lambda y: 0.8 * torch.sigmoid(3 * y)
    q, tau, t = particle_quadrature(mu, sig, om, tau_fn, 0.2, 3.0, 3, lambda t: t - 2.5)
    tr = torch.exp(-tau)
    sig_bar = (tau[:, 1:] - tau[:, :-1]) / (t[:, 1:] - t[:, :-1])
    sig_i = om[:, None] * torch.exp(-(t[:, :-1] - mu[:, None]) ** 2 / (2 * sig[:, None] ** 2))
    lit = ((tr[:, :-1] - tr[:, 1:]) * sig_i / sig_bar).sum(-1)
    assert torch.allclose(q, lit, rtol=1e-12)


def test_quadrature_converges_to_volume_rendering_with_exact_tau():
    """With the exact optical depth in place of the bounds, sum_i q_i tends to
    int T sigma_i dt (the emission integral of Eq. 2) as N grows."""
    tn = 0.2
    mus = np.array([2.0, 2.3, 3.0])
    sig = np.array([0.3, 0.2, 0.5])
    om = np.array([1.5, 2.0, 0.8])

    def tau_exact(t):
        tt = t[..., None]
        return (_t(om * sig) * math.sqrt(math.pi / 2)
                * (torch.special.erf((tt - _t(mus)) / (math.sqrt(2) * _t(sig)))
                   - torch.special.erf((tn - _t(mus)) / (math.sqrt(2) * _t(sig))))).sum(-1)

    def emission(i):
        f = lambda t: math.exp(-tau_exact(_t([t])).item()) * om[i] * math.exp(
            -(t - mus[i]) ** 2 / (2 * sig[i] ** 2))
        return integrate.quad(f, tn, 20, limit=200)[0]

    ref = np.array([emission(i) for i in range(3)])
    errs = []
    for n in (3, 31, 255):
        q, _, _ = particle_quadrature(_t(mus), _t(sig), _t(om), tau_exact, tn, 3.0, n, lambda t: t)
        errs.append(np.abs(q.numpy() - ref).max())
    # the left-edge rule converges at first order in 1/N
    assert errs[2] < errs[1] < errs[0]
    assert errs[2] < 6e-3


# ---------------------------------------------------------------------------
# Screen proxy (App. D).
# ---------------------------------------------------------------------------

def _single_gaussian_scene(mean, scale, quat, w, rgb=(1.0, 0.5, 0.25)):
    return W.Scene(np.array([mean], np.float32), np.array([scale], np.float32),
                   np.array([quat], np.float32), np.array([w], np.float32),
                   np.array([rgb], np.float32), -1)


def test_proxy_isotropic_on_axis_closed_form():
    cam = W.camera_on_axis(0.0, 200, 160)
    dist, s, w, c = 5.0, float(np.float32(0.2)), 3.0, 0.01  # inputs are float32
    scene = _single_gaussian_scene([0, 0, dist], [s, s, s], [1, 0, 0, 0], w)
    p = screen_proxy(scene_tensors(scene), cam, c)
    big_c = -math.log(1 - c) / (s * math.sqrt(2 * math.pi))
    sin2 = 2 * s * s / dist ** 2 * math.log(w / big_c)
    r = cam.fx * math.sqrt(sin2 / (1 - sin2))
    assert p.valid.item()
    assert np.allclose(p.mean2d[0].numpy(), [cam.cx, cam.cy], atol=1e-9)
    assert np.allclose(p.half[0].numpy(), [r, r], rtol=1e-9)


def test_proxy_boundary_is_the_level_set_omega_equals_c():
    """Points on the ellipse satisfy w exp(K(d)) = C (the conic of Eq. 17)."""
    cam = W.camera_on_axis(0.0, 320, 240)
    rng = np.random.default_rng(5)
    for _ in range(10):
        mean = [rng.uniform(-0.5, 0.5), rng.uniform(-0.4, 0.4), rng.uniform(3, 6)]
        scale = np.exp(rng.normal(-1.5, 0.4, 3))
        quat = rng.normal(size=4)
        w = rng.lognormal(1.0, 0.5)
        scene = _single_gaussian_scene(mean, scale, quat, w)
        st = scene_tensors(scene)
        p = screen_proxy(st, cam, 0.01)
        if not p.valid.item():
            continue
        # the check uses the float32-rounded inputs the oracle saw
        mean, scale, quat, w = (np.asarray(v, np.float64) for v in
                                (scene.means[0], scene.scales[0], scene.quats[0], scene.densities[0]))
        mu_c = np.array(mean)
        rot = quat_to_rot(_t(quat)).numpy()
        prec = rot @ np.diag(1 / scale ** 2) @ rot.T
        u = mu_c / np.linalg.norm(mu_c)
        big_c = -math.log(0.99) * math.sqrt(u @ prec @ u) / math.sqrt(2 * math.pi)
        sig2d = (p.axes[0].T @ torch.diag(p.half[0] ** 2) @ p.axes[0]).numpy()
        ev, evec = np.linalg.eigh(sig2d)
        for ang in np.linspace(0, 2 * np.pi, 9)[:-1]:
            pt = p.mean2d[0].numpy() + evec @ (np.sqrt(ev) * [math.cos(ang), math.sin(ang)])
            d = np.array([(pt[0] - cam.cx) / cam.fx, (pt[1] - cam.cy) / cam.fy, 1.0])
            d /= np.linalg.norm(d)
            _, _, om = ray_gaussian(_t(np.zeros(3)), _t(d), _t(mu_c), _t(rot), _t(scale), _t(w))
            assert om.item() == pytest.approx(big_c, rel=1e-7)


def test_proxy_covers_the_opacity_level_set():
    """Pixels whose exact single-Gaussian opacity 1 - exp(-tau_bar) reaches c
    lie inside the rectangle (the paper calls the proxy conservative but
    'not a strict upper bound'; allow a small violation rate)."""
    cam = W.camera_on_axis(0.0, 160, 120)
    rng = np.random.default_rng(9)
    bad = total = 0
    for _ in range(8):
        mean = [rng.uniform(-0.3, 0.3), rng.uniform(-0.2, 0.2), rng.uniform(2.5, 4)]
        scale = np.exp(rng.normal(-2.0, 0.5, 3))
        quat = rng.normal(size=4)
        w = rng.lognormal(1.5, 0.5)
        scene = _single_gaussian_scene(mean, scale, quat, w)
        st = scene_tensors(scene)
        p = screen_proxy(st, cam, 0.01)
        ys, xs = np.mgrid[0:cam.height, 0:cam.width]
        px, py = torch.as_tensor(xs.ravel()), torch.as_tensor(ys.ravel())
        d = oracle.pixel_directions(cam, px, py)
        rot = quat_to_rot(st["quats"]).expand(d.shape[0], 3, 3)
        mu, sig, om = ray_gaussian(torch.zeros(3, dtype=DT), d, st["means"].expand(d.shape[0], 3),
                                   rot, st["scales"].expand(d.shape[0], 3), st["densities"].expand(d.shape[0]))
        m0 = particle_moments(mu, sig, om, cam.t_near, 0, 0.0, 1.0)[:, 0]
        opaque = (1 - torch.exp(-m0)) >= 0.01
        from oracle.proxy import rect_margin
        inside = rect_margin(p, torch.zeros_like(px), px, py) >= 0
        bad += int((opaque & ~inside).sum())
        total += int(opaque.sum())
    assert total > 100
    assert bad <= 0.02 * total


def _fibonacci_sphere(n):
    k = np.arange(n) + 0.5
    z = 1 - 2 * k / n
    phi = math.pi * (1 + math.sqrt(5)) * k
    rxy = np.sqrt(1 - z * z)
    return np.stack([rxy * np.cos(phi), rxy * np.sin(phi), z], -1)


def _off_centre_rotated_camera():
    cam = W.camera_look_at((2.0, -1.0, -6.0), (0.3, 0.2, 0.0), (0.1, 1.0, 0.2), 320, 200)
    return dataclasses.replace(cam, cx=0.3 * cam.width, cy=0.62 * cam.height)


def test_bounding_sphere_cull_against_sampled_sphere():
    """Sec. 3.3 culls with the bounding sphere (mean, max s): keep a Gaussian
    iff some point of that sphere projects into the image in front of t_n
    (tested away from the frustum's edges, where the plane test is exact),
    and, reading R14, the centre itself lies beyond t_n. Spheres straddle,
    touch and miss each of the four side planes and the near plane of a
    rotated camera with an off-centre principal point."""
    cam = _off_centre_rotated_camera()
    r_wc = cam.world_to_cam[:, :3].astype(np.float64)
    t_wc = cam.world_to_cam[:, 3].astype(np.float64)
    fx, fy, cx, cy, wd, ht, tn = cam.fx, cam.fy, cam.cx, cam.cy, cam.width, cam.height, cam.t_near
    z0, rad = 4.0, 0.1
    # a point in the middle of each side face (camera frame) and the face's
    # inward unit normal, built from the image borders u = 0, u = W, v = 0, v = H
    mid_u, mid_v = (wd / 2 - cx) / fx, (ht / 2 - cy) / fy
    faces = [(np.array([-cx / fx, mid_v, 1.0]) * z0, np.array([fx, 0.0, cx])),
             (np.array([(wd - cx) / fx, mid_v, 1.0]) * z0, np.array([-fx, 0.0, wd - cx])),
             (np.array([mid_u, -cy / fy, 1.0]) * z0, np.array([0.0, fy, cy])),
             (np.array([mid_u, (ht - cy) / fy, 1.0]) * z0, np.array([0.0, -fy, ht - cy]))]
    centres = []
    for p0, n in faces:
        n = n / np.linalg.norm(n)
        for d in (-1.5, -1.03, -0.97, -0.5, 0.5):
            centres.append(p0 + d * rad * n)
    for d in (-1.5, -1.03, -0.97, -0.5, 0.5, 1.5):
        centres.append(np.array([mid_u * tn, mid_v * tn, tn]) + np.array([0.0, 0.0, d * rad]))
    centres = np.array(centres)
    sphere = _fibonacci_sphere(40000)
    expected = []
    for c in centres:
        pts = c + rad * sphere
        z = pts[:, 2]
        with np.errstate(divide="ignore", invalid="ignore"):
            u = fx * pts[:, 0] / z + cx
            v = fy * pts[:, 1] / z + cy
        seen = (z > tn) & (u >= 0) & (u <= wd) & (v >= 0) & (v <= ht)
        expected.append(bool(seen.any()) and c[2] > tn)
    means = (centres - t_wc) @ r_wc  # world = R^T (camera - t)
    n = len(centres)
    rng = np.random.default_rng(3)
    scene = W.Scene(means.astype(np.float32),
                    np.tile(np.array([[rad, rad / 2, rad / 3]], np.float32), (n, 1)),
                    rng.normal(size=(n, 4)).astype(np.float32), np.ones(n, np.float32),
                    np.ones((n, 3), np.float32), -1)
    got = screen_proxy(scene_tensors(scene), cam, 0.01).in_frustum.numpy()
    assert sum(expected) not in (0, n)
    assert got.tolist() == expected


def test_pixel_rays_of_a_rotated_camera_pass_through_projected_points():
    """Sec. 3.3 maps pixel p to the ray direction normalize(K^-1 p) in camera
    space: the ray through the projection of a world point under K [R | t]
    (here at a continuous pixel position) passes through that point."""
    cam = _off_centre_rotated_camera()
    # an exactly orthonormal (float64) rotation: the float32 one is orthonormal
    # only to 3e-8, which would hide nothing but blur the bound below
    u_, _, vt_ = np.linalg.svd(cam.world_to_cam[:, :3].astype(np.float64))
    r_wc = u_ @ vt_
    t_wc = cam.world_to_cam[:, 3].astype(np.float64)
    cam.world_to_cam = np.concatenate([r_wc, t_wc[:, None]], 1)
    assert np.abs(r_wc - r_wc.T).max() > 0.1  # R and R^T differ
    rng = np.random.default_rng(8)
    pts = rng.uniform(-1.5, 1.5, size=(50, 3))
    xc = pts @ r_wc.T + t_wc
    u = cam.fx * xc[:, 0] / xc[:, 2] + cam.cx
    v = cam.fy * xc[:, 1] / xc[:, 2] + cam.cy
    d = oracle.pixel_directions(cam, _t(u - 0.5), _t(v - 0.5)).numpy()
    o = cam.origin
    to_pt = pts - o
    cross = np.cross(to_pt, d)
    assert np.abs(np.linalg.norm(d, axis=1) - 1).max() < 1e-14
    assert (np.einsum("ni,ni->n", to_pt, d) > 0).all()
    assert (np.linalg.norm(cross, axis=1) / np.linalg.norm(to_pt, axis=1)).max() < 1e-12


def test_proxy_axes_follow_the_ellipse_and_a_circle_takes_the_x_axis():
    """The rectangle's first axis is the projected ellipse's major axis: a
    prolate Gaussian on the optical axis turned by phi about it projects to an
    ellipse whose major axis makes the angle phi with the image x axis. A
    sphere on the axis projects to a circle, which takes the x axis (the
    orientation reading for a circle)."""
    cam = W.camera_on_axis(0.0, 200, 160)
    for phi in (0.3, 1.2, 2.0, -0.7):
        q = [math.cos(phi / 2), 0.0, 0.0, math.sin(phi / 2)]
        scene = _single_gaussian_scene([0, 0, 5.0], [0.3, 0.06, 0.05], q, 4.0)
        p = screen_proxy(scene_tensors(scene), cam, 0.01)
        e1 = p.axes[0, 0].numpy()
        assert abs(abs(e1 @ [math.cos(phi), math.sin(phi)]) - 1) < 1e-12
        assert p.half[0, 0] > 2 * p.half[0, 1]
        assert abs(p.axes[0, 1].numpy() @ e1) < 1e-15
    scene = _single_gaussian_scene([0, 0, 5.0], [0.2, 0.2, 0.2], [1, 0, 0, 0], 4.0)
    p = screen_proxy(scene_tensors(scene), cam, 0.01)
    assert p.axes[0].numpy().tolist() == [[1.0, 0.0], [-0.0, 1.0]]


# ---------------------------------------------------------------------------
# Spherical harmonics against scipy's complex harmonics.
# ---------------------------------------------------------------------------

def test_real_sh_against_scipy():
    rng = np.random.default_rng(1)
    d = rng.normal(size=(50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    got = real_sh_basis(_t(d), 3).numpy()
    theta = np.arccos(d[:, 2])
    phi = np.arctan2(d[:, 1], d[:, 0])
    for l in range(4):
        for m in range(-l, l + 1):
            y = sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                ref = math.sqrt(2) * (-1) ** m * y.real
            elif m < 0:
                ref = math.sqrt(2) * (-1) ** m * y.imag
            else:
                ref = y.real
            assert np.allclose(got[:, l * l + l + m], ref, atol=1e-12)


# ---------------------------------------------------------------------------
# Whole-pipeline pins.
# ---------------------------------------------------------------------------

def _tiny_scene(seed=0, n=6, rgb=None):
    rng = np.random.default_rng(seed)
    means = rng.normal(0, 0.15, (n, 3))
    scales = np.exp(rng.normal(-1.8, 0.3, (n, 3)))
    quats = rng.normal(size=(n, 4))
    quats /= np.linalg.norm(quats, axis=1, keepdims=True)
    dens = rng.lognormal(1.0, 0.5, n)
    colors = rng.uniform(0, 1, (n, 3)) if rgb is None else np.tile(rgb, (n, 1))
    return W.Scene(means.astype(np.float32), scales.astype(np.float32), quats.astype(np.float32),
                   dens.astype(np.float32), colors.astype(np.float32), -1)


@pytest.mark.parametrize("k_mom", [4, 6, 8])
def test_single_colour_scene_renders_exact_opacity(k_mom):
    """S = c O when every Gaussian has colour c, so Eq. 15 gives exactly
    c (1 - e^-m0) + e^-m0 bg, and m0 is the exact optical depth: compare
    with brute-force ray marching of the summed 3D density."""
    colour = np.array([0.9, 0.4, 0.2])
    scene = _tiny_scene(1, 8, rgb=colour)
    cam = W.camera_on_axis(2.0, 24, 20)
    cam.background = (0.1, 0.2, 0.3)
    opts = W.Options(n_moments=k_mom, full_coverage=True)
    r = oracle.render_image(scene, cam, opts)
    st = scene_tensors(scene)
    rot = quat_to_rot(st["quats"]).numpy()
    precs = [rot[i] @ np.diag(1 / scene.scales[i].astype(float) ** 2) @ rot[i].T for i in range(scene.n)]
    for pix in [0, 55, 201, 333, 479]:
        px, py = pix % cam.width, pix // cam.width
        d = oracle.pixel_directions(cam, torch.tensor([px]), torch.tensor([py]))[0].numpy()
        o = cam.origin

        def dens(t):
            x = o + t * d
            return sum(scene.densities[i] * math.exp(-0.5 * (x - scene.means[i]) @ precs[i]
                                                     @ (x - scene.means[i])) for i in range(scene.n))

        centres = sorted(float((scene.means[i] - o) @ d) for i in range(scene.n))
        with warnings.catch_warnings():
            # quad reports round-off near its tolerance floor; the bar below
            # (1e-7 relative) is far above it
            warnings.simplefilter("ignore", integrate.IntegrationWarning)
            tau = integrate.quad(dens, cam.t_near, 50, limit=800, epsabs=1e-15, epsrel=1e-10,
                                 points=centres)[0]
        assert r["moments"][pix, 0] == pytest.approx(tau, rel=1e-7, abs=1e-13)
        assert r["opacity"][pix] >= opts.eps
        expect = colour * (1 - math.exp(-tau)) + math.exp(-tau) * np.array(cam.background)
        assert np.allclose(r["image"][pix], expect, atol=1e-9)


def test_single_gaussian_renders_eq16_opacity():
    scene = _tiny_scene(2, 1, rgb=np.array([1.0, 1.0, 1.0]))
    cam = W.camera_on_axis(2.0, 16, 16)
    opts = W.Options(full_coverage=True)
    r = oracle.render_image(scene, cam, opts)
    op = -np.expm1(-r["moments"][:, 0])
    ok = r["opacity"] >= opts.eps
    assert ok.sum() > 100
    assert np.allclose(r["image"][ok, 0], op[ok], rtol=1e-12, atol=1e-15)
    # where O < eps Eq. 15 divides by eps instead
    assert np.allclose(r["image"][~ok, 0], op[~ok] * r["s_rgb"][~ok, 0] / opts.eps, rtol=1e-12, atol=1e-300)


def test_image_is_invariant_to_gaussian_order():
    scene, cams, opts = W.w1_small()
    sub = scene.subset(np.arange(300))
    perm = np.random.default_rng(0).permutation(300)
    pix = np.arange(0, 128 * 128, 7)
    a = oracle.render_image(sub, cams[0], opts, pixels=pix)
    b = oracle.render_image(sub.subset(perm), cams[0], opts, pixels=pix)
    assert np.abs(a["image"] - b["image"]).max() < 1e-12


def test_far_separated_narrow_gaussians_composite_front_to_back():
    """Two thin Gaussians far apart along the ray: the moment bounds become
    step functions (atom limit), giving front-to-back compositing
    c_A a_A + (1 - a_A) c_B a_B."""
    means = np.array([[0, 0, 1.0], [0, 0, 6.0]], np.float32)
    scales = np.array([[0.3, 0.3, 0.01], [0.3, 0.3, 0.01]], np.float32)
    quats = np.array([[1, 0, 0, 0], [1, 0, 0, 0]], np.float32)
    dens = np.array([40.0, 60.0], np.float32)
    cols = np.array([[1, 0, 0], [0, 0, 1]], np.float32)
    scene = W.Scene(means, scales, quats, dens, cols, -1)
    cam = W.camera_on_axis(2.0, 8, 8)
    r = oracle.render_image(scene, cam, W.Options(n_moments=4), pixels=[4 * 8 + 4])
    d = oracle.pixel_directions(cam, torch.tensor([4]), torch.tensor([4]))[0].numpy()
    o = cam.origin

    def depth(i):  # optical depth of Gaussian i alone along the pixel ray
        prec = np.diag(1.0 / scales[i].astype(float) ** 2)
        f = lambda t: dens[i] * math.exp(-0.5 * (o + t * d - means[i]) @ prec @ (o + t * d - means[i]))
        tc = float((means[i] - o) @ d)
        return integrate.quad(f, tc - 1, tc + 1, points=[tc], epsabs=1e-14)[0]

    m_a, m_b = depth(0), depth(1)
    assert r["moments"][0, 0] == pytest.approx(m_a + m_b, rel=1e-7)
    a_a, a_b = 1 - math.exp(-m_a), 1 - math.exp(-m_b)
    ref = np.array([1, 0, 0]) * a_a + (1 - a_a) * np.array([0, 0, 1]) * a_b
    assert np.abs(r["image"][0] - ref).max() < 2e-3


def test_multicolour_image_close_to_ray_marched_vre():
    """Quality check only (the method approximates Eq. 2): on a tiny scene the
    image is near a fine ray marching of the volume rendering equation."""
    scene = _tiny_scene(3, 5)
    cam = W.camera_on_axis(2.0, 12, 12)
    r = oracle.render_image(scene, cam, W.Options(n_moments=6, full_coverage=True))
    st = scene_tensors(scene)
    rot = quat_to_rot(st["quats"]).numpy()
    precs = [rot[i] @ np.diag(1 / scene.scales[i].astype(float) ** 2) @ rot[i].T for i in range(scene.n)]
    t = np.linspace(cam.t_near, 6, 20001)
    err = []
    for pix in range(0, 144, 5):
        px, py = pix % 12, pix // 12
        d = oracle.pixel_directions(cam, torch.tensor([px]), torch.tensor([py]))[0].numpy()
        x = cam.origin + t[:, None] * d
        sig = np.stack([scene.densities[i] * np.exp(-0.5 * np.einsum(
            "ti,ij,tj->t", x - scene.means[i], precs[i], x - scene.means[i])) for i in range(scene.n)])
        tot = sig.sum(0)
        tau = np.concatenate([[0], np.cumsum(0.5 * (tot[1:] + tot[:-1]) * np.diff(t))])
        em = (np.exp(-tau) * (sig.T @ scene.colors).T).T
        ref = np.trapezoid(em, t, axis=0)
        err.append(np.abs(ref - r["image"][pix]).max())
    assert max(err) < 0.1


# ---------------------------------------------------------------------------
# Gradients: float64 autograd of the oracle vs central finite differences.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("basis,k_mom", [("power", 4), ("trigonometric", 4), ("trigonometric", 6)])
def test_oracle_gradients_vs_central_differences(basis, k_mom):
    """Autograd through the whole oracle render (for the trigonometric basis
    also through the Toeplitz solves and the kernel polynomial's roots on the
    circle) against central differences of its image."""
    scene = _tiny_scene(4, 4)
    scene.colors = np.random.default_rng(4).normal(0, 0.3, (4, 4, 3)).astype(np.float32)
    scene.sh_degree = 1
    cam = W.camera_on_axis(2.0, 8, 8)
    opts = W.Options(n_moments=k_mom, full_coverage=True)
    opts.basis = basis
    g_img = np.random.default_rng(5).normal(size=(64, 3))
    grads = oracle.render_backward(scene, cam, opts, g_img)

    def loss(sc):
        img = oracle.render_image(sc, cam, opts)["image"]
        return float((img * g_img).sum())

    base = {k: np.asarray(getattr(scene, k), np.float64) for k in oracle.render.PARAMS}

    def loss64(params):
        # the oracle promotes float32 inputs; feed float64 through a shallow scene copy
        sc = W.Scene(params["means"], params["scales"], params["quats"], params["densities"],
                     params["colors"], scene.sh_degree)
        return loss(sc)

    rng = np.random.default_rng(6)
    for name in oracle.render.PARAMS:
        arr = base[name]
        for _ in range(3):
            idx = tuple(rng.integers(0, s) for s in arr.shape)
            h = 1e-6 * max(1.0, abs(arr[idx]))
            p = {k: v.copy() for k, v in base.items()}
            p[name][idx] += h
            lp = loss64(p)
            p[name][idx] -= 2 * h
            lm = loss64(p)
            fd = (lp - lm) / (2 * h)
            assert grads[name][idx] == pytest.approx(fd, rel=1e-5, abs=1e-8), name


def test_linearisation_point():
    """App. C expands the warp at the particle mean; for a mean before the near
    bound the expansion point is t_n (reading), continued linearly to mu."""
    tn, c, s = 0.2, 0.3, 0.05
    for mu in (0.5, 3.0, 11.0):
        g, gp = linearised_warp(_t([mu]), tn, _t([c]), _t([s]))
        assert g.item() == pytest.approx((warp(mu, tn) - c) / s, rel=1e-14)
        assert gp.item() == pytest.approx(warp_prime(mu, tn) / s, rel=1e-14)
    mu = -0.4
    g, gp = linearised_warp(_t([mu]), tn, _t([c]), _t([s]))
    assert gp.item() == pytest.approx(warp_prime(tn, tn) / s, rel=1e-14)
    assert g.item() == pytest.approx((warp(tn, tn) - c) / s + gp.item() * (mu - tn), rel=1e-14)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_bounds_invariant_under_affine_moment_variable(n):
    """The canonical representation maps onto itself under y' = (y - a)/b,
    b > 0, so tau(eta) computed from transformed moments at the transformed
    query is unchanged (the oracle's per-pixel moment variable relies on it)."""
    rng = np.random.default_rng(n + 20)
    grid = np.linspace(-2, 2, 4001)
    dens = sum(rng.uniform(0.2, 1) * np.exp(-(grid - rng.uniform(-1, 1)) ** 2 / rng.uniform(0.01, 0.2))
               for _ in range(3))
    dens *= 0.7 / dens.sum()
    a, bsc = 0.37, 2.5
    y2 = (grid - a) / bsc
    m1 = _t([(dens * grid ** k).sum() for k in range(2 * n + 1)])
    m2 = _t([(dens * y2 ** k).sum() for k in range(2 * n + 1)])
    etas = np.linspace(-1.8, 1.8, 25)
    t1, _, _ = bound_tau(m1[None].expand(25, -1), _t(etas), n, 0.25)
    t2, _, _ = bound_tau(m2[None].expand(25, -1), _t((etas - a) / bsc), n, 0.25)
    assert torch.allclose(t1, t2, atol=1e-10)


# ---------------------------------------------------------------------------
# Surrogate reference (not in the paper): pinned to finite differences and to
# torch float64 autograd of the same network.
# ---------------------------------------------------------------------------

def _mlp_batch(n, seed):
    rng = np.random.default_rng(seed)
    x = np.concatenate([rng.normal(0, 1, (n, 6)), rng.uniform(-4, 4, (n, 1)),
                        rng.uniform(0.05, 3, (n, 1))], axis=1)
    t = rng.uniform(0, 1, n)
    return x, t


def test_surrogate_reference_gradient_vs_finite_differences():
    from oracle import surrogate as S
    theta = S.init_params(3)
    x, t = _mlp_batch(40, 4)
    loss, g = S.loss_grad(theta, x, t, bf16_mode=False)
    rng = np.random.default_rng(5)
    for i in rng.choice(S.N_PARAMS, 25, replace=False):
        h = 1e-6
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (S.loss_grad(tp, x, t, False)[0] - S.loss_grad(tm, x, t, False)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-10)


def test_surrogate_reference_vs_torch_autograd():
    from oracle import surrogate as S
    theta = S.init_params(7)
    x, t = _mlp_batch(64, 8)
    loss, g = S.loss_grad(theta, x, t, bf16_mode=False)
    th = torch.tensor(theta, requires_grad=True)
    p, o = {}, 0
    for k, s in S.SIZES.items():
        n = int(np.prod(s))
        p[k] = th[o:o + n].reshape(s)
        o += n
    xt = torch.tensor(x)
    gelu = lambda v: 0.5 * v * (1 + torch.tanh(S.GELU_C * (v + S.GELU_A * v ** 3)))
    a1 = gelu(xt[:, :7] @ p["W1"].T + p["b1"])
    a2 = gelu(a1 @ p["W2"].T + p["b2"])
    f = torch.sigmoid(a2 @ p["w3"] + p["b3"][0])
    lt = ((torch.exp(-xt[:, 7] * f) - torch.tensor(t)) ** 2).mean()
    lt.backward()
    assert float(lt.detach()) == pytest.approx(loss, rel=1e-12)
    assert np.allclose(th.grad.numpy(), g, rtol=1e-9, atol=1e-14)


def test_surrogate_input_gradient_vs_finite_differences():
    """dF/d(inputs) without rounding against central differences of F."""
    from oracle import surrogate as S
    theta = S.init_params(9)
    x, _ = _mlp_batch(30, 10)
    f, dx = S.input_grad(theta, x, bf16_mode=False)
    assert np.array_equal(f, S.forward(theta, x, bf16_mode=False)[0])
    h = 1e-6
    for k in range(7):
        xp = x.copy(); xp[:, k] += h
        xm = x.copy(); xm[:, k] -= h
        fd = (S.forward(theta, xp, False)[0] - S.forward(theta, xm, False)[0]) / (2 * h)
        assert np.allclose(dx[:, k], fd, rtol=1e-6, atol=1e-10)


def test_surrogate_input_gradient_rounding_points():
    """With the kernels' rounding points: F is the bf16 forward value, and the
    gradient is the exact one up to the bf16 rounding of dZ2 and dZ1 (unit
    roundoff 2^-9 each, accumulated over 64 terms)."""
    from oracle import surrogate as S
    theta = S.init_params(11)
    x, _ = _mlp_batch(200, 12)
    f, dx = S.input_grad(theta, x, bf16_mode=True)
    assert np.array_equal(f, S.forward(theta, x, bf16_mode=True)[0])
    xt = torch.tensor(x[:, :7], requires_grad=True)
    S.forward_torch(theta, xt).sum().backward()
    ref = xt.grad.numpy()
    rel = np.linalg.norm(dx - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert np.median(rel) < 3e-3 and rel.max() < 3e-2
    # and not equal: the rounding points are there
    assert rel.max() > 0


def test_surrogate_tau_model_gradient_vs_finite_differences():
    """The feature map's derivative: d tau / d(moments, query) of the torch
    hook (no rounding) against central differences of the numpy model."""
    from oracle import surrogate as S
    theta = S.init_params(13)
    rng = np.random.default_rng(14)
    n = 12
    mom = np.empty((n, 7))
    # moments of small positive measures on [-1, 1] (the renderer's moment
    # variable is standardised per pixel, so its moments are of this kind)
    for i in range(n):
        pts = rng.uniform(-1, 1, 5)
        w = rng.uniform(0.1, 1, 5)
        mom[i] = [(w * pts ** k).sum() for k in range(7)]
    y = rng.uniform(-0.8, 0.8, n)
    mt = torch.tensor(mom, requires_grad=True)
    yt = torch.tensor(y, requires_grad=True)
    tau = S.tau_model_torch(theta, network="exact")(mt, yt)
    ref = S.tau_model(theta, bf16_mode=False)(mom, y).numpy()
    assert np.allclose(tau.detach().numpy(), ref, rtol=1e-12)
    gm, gy = torch.autograd.grad(tau.sum(), [mt, yt])
    model = S.tau_model(theta, False)

    def fd(shift, h):
        # central differences, Richardson-extrapolated (the feature map is
        # steep where the measure's variance is small)
        d = lambda hh: (model(*shift(hh)).numpy() - model(*shift(-hh)).numpy()) / (2 * hh)
        return (4 * d(h / 2) - d(h)) / 3
    for k in range(7):
        def shift(hh, k=k):
            m = mom.copy()
            m[:, k] += hh
            return m, y
        ref_k = fd(shift, 1e-6 * np.abs(mom[:, k]).max())
        assert np.allclose(gm[:, k].numpy(), ref_k, rtol=1e-6, atol=1e-7 * np.abs(ref_k).max())
    ref_y = fd(lambda hh: (mom, y + hh), 1e-6)
    assert np.allclose(gy.numpy(), ref_y, rtol=1e-6, atol=1e-9)


def test_bf16_rounding_is_nearest_even():
    from oracle.surrogate import bf16
    assert bf16(1.0) == 1.0
    assert bf16(1.0 + 2 ** -8) == 1.0          # tie -> even
    assert bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6  # tie -> even (up)
    assert bf16(1.0 + 2 ** -8 + 2 ** -12) == 1.0 + 2 ** -7


# ---------------------------------------------------------------------------
# Ground truth of Eqs. 2-3 (oracle.exact) used for image quality.
# ---------------------------------------------------------------------------

def test_exact_single_gaussian_closed_form():
    """One Gaussian: int sigma T dt = 1 - T(inf), so L = c (1 - e^-tau) + e^-tau bg."""
    from oracle.exact import exact_ray
    mu, sig, om = np.array([3.0]), np.array([0.2]), np.array([4.0])
    tau = om[0] * sig[0] * math.sqrt(math.pi / 2) * erfc((0.5 - mu[0]) / (math.sqrt(2) * sig[0]))
    c = np.array([[0.7, 0.2, 0.1]])
    bg = np.array([0.3, 0.3, 0.9])
    got = exact_ray(mu, sig, om, c, 0.5, bg)
    assert np.allclose(got, c[0] * (1 - math.exp(-tau)) + math.exp(-tau) * bg, atol=1e-12)
    # a Gaussian cut by the near bound
    got = exact_ray(np.array([0.6]), sig, om, c, 0.5, bg)
    tau = om[0] * sig[0] * math.sqrt(math.pi / 2) * erfc((0.5 - 0.6) / (math.sqrt(2) * sig[0]))
    assert np.allclose(got, c[0] * (1 - math.exp(-tau)) + math.exp(-tau) * bg, atol=1e-12)


def test_exact_grey_scene_and_front_to_back_limit():
    """Equal colours: L = c (1 - T(inf)) for any overlap. Far-apart thin
    Gaussians: front-to-back compositing of their opacities."""
    from oracle.exact import exact_ray
    rng = np.random.default_rng(11)
    mu = rng.uniform(1, 3, 12)
    sig = rng.uniform(0.01, 0.4, 12)
    om = rng.lognormal(0, 1, 12)
    c = np.tile([0.5, 0.25, 1.0], (12, 1))
    tot = (om * sig * math.sqrt(math.pi / 2) * erfc((0.2 - mu) / (math.sqrt(2) * sig))).sum()
    got = exact_ray(mu, sig, om, c, 0.2, np.zeros(3))
    assert np.allclose(got, c[0] * (1 - math.exp(-tot)), rtol=1e-9)
    mu2, sig2, om2 = np.array([2.0, 5.0]), np.array([0.05, 0.05]), np.array([10.0, 20.0])
    a = 1 - np.exp(-om2 * sig2 * math.sqrt(2 * math.pi))
    c2 = np.array([[1.0, 0, 0], [0, 0, 1.0]])
    got = exact_ray(mu2, sig2, om2, c2, 0.2, np.zeros(3))
    assert np.allclose(got, c2[0] * a[0] + (1 - a[0]) * c2[1] * a[1], atol=1e-12)


def test_exact_pixels_match_ray_marching_of_3d_density():
    """The whole chain (rays, Eqs. 4-6, SH colour, Eqs. 2-3) against a fine
    ray marching of the summed 3D density of a tiny multicolour scene."""
    from oracle.exact import exact_pixels
    scene = _tiny_scene(3, 5)
    cam = W.camera_on_axis(2.0, 12, 12)
    pix = np.arange(0, 144, 7)
    got = exact_pixels(scene, cam, pix)
    st = scene_tensors(scene)
    rot = quat_to_rot(st["quats"]).numpy()
    precs = [rot[i] @ np.diag(1 / scene.scales[i].astype(float) ** 2) @ rot[i].T for i in range(scene.n)]
    t = np.linspace(cam.t_near, 6, 200001)
    for k, p in enumerate(pix):
        d = oracle.pixel_directions(cam, torch.tensor([p % 12]), torch.tensor([p // 12]))[0].numpy()
        x = cam.origin + t[:, None] * d
        sig = np.stack([scene.densities[i] * np.exp(-0.5 * np.einsum(
            "ti,ij,tj->t", x - scene.means[i], precs[i], x - scene.means[i])) for i in range(scene.n)])
        tot = sig.sum(0)
        tau = np.concatenate([[0], np.cumsum(0.5 * (tot[1:] + tot[:-1]) * np.diff(t))])
        ref = np.trapezoid((np.exp(-tau) * (sig.T @ scene.colors).T).T, t, axis=0)
        assert np.abs(ref - got[k]).max() < 2e-6, p


# ---------------------------------------------------------------------------
# Inputs of the learned surrogate (oracle.surrogate.features / query).
# ---------------------------------------------------------------------------

def _normal_raw_moments(m, s, k_max=6):
    from scipy.stats import norm
    return np.array([norm(m, s).moment(k) if k else 1.0 for k in range(k_max + 1)])


def test_surrogate_features_of_a_normal_measure():
    """Any normal measure standardises to the moments 0, 1, 0, 3, 0, 15."""
    from oracle.surrogate import features, query
    mom = np.stack([2.5 * _normal_raw_moments(1.7, 0.4), 0.1 * _normal_raw_moments(-3.0, 2.0)])
    feat, mean, std = features(mom)
    assert np.allclose(feat, np.arcsinh([0, 1, 0, 3, 0, 15])[None, :], atol=1e-9)
    assert np.allclose(mean, [1.7, -3.0]) and np.allclose(std, [0.4, 2.0])
    assert np.allclose(query(np.array([1.7 + 0.8, -3.0 - 30]), mean, std), [2.0, -10.0])


def test_surrogate_features_invariant_under_affine_variable():
    """Features and standardised queries of an atomic measure do not change
    when the moment variable is mapped by y -> a y + c, a > 0."""
    from oracle.surrogate import features, query
    rng = np.random.default_rng(12)
    x = rng.normal(size=5)
    w = rng.uniform(0.1, 1.0, 5)
    a, c = 2.7, -1.3
    m1 = np.array([[(w * x ** k).sum() for k in range(7)]])
    m2 = np.array([[(w * (a * x + c) ** k).sum() for k in range(7)]])
    f1, mu1, s1 = features(m1)
    f2, mu2, s2 = features(m2)
    assert np.allclose(f1, f2, atol=1e-9)
    assert np.allclose(query(0.3, mu1, s1), query(a * 0.3 + c, mu2, s2))
    # direct definition: standardised moments of the atoms
    z = (x - (w * x).sum() / w.sum())
    z = z / math.sqrt((w * z * z).sum() / w.sum())
    assert np.allclose(f1[0], np.arcsinh([(w * z ** k).sum() / w.sum() for k in range(1, 7)]))


def test_render_through_the_surrogate_inputs_reproduces_the_plain_render():
    """The reconstruction written as a function of the network's inputs alone
    (exact_model, no clamp) renders the same image as the plain path, so the
    inputs carry everything the bounds use."""
    from oracle.surrogate import exact_model
    scene, cams, opts = W.w1_small()
    opts.n_moments = 6
    sub = scene.subset(np.arange(400))
    pix = np.arange(0, 128 * 128, 37)
    a = oracle.render_image(sub, cams[0], opts, pixels=pix)
    b = oracle.render_image(sub, cams[0], opts, pixels=pix, tau_model=exact_model(opts.beta, np.inf))
    assert a["n_pairs"] > 500
    assert np.abs(a["image"] - b["image"]).max() < 1e-8


# ---------------------------------------------------------------------------
# Consistency penalty (App. E, regularisation).
# ---------------------------------------------------------------------------

def test_interval_depth_is_the_integral_of_the_particle_density():
    from oracle.quadrature import interval_depth
    rng = np.random.default_rng(21)
    mu, sig, om = rng.uniform(1, 3, 6), rng.uniform(0.05, 0.5, 6), rng.lognormal(0, 1, 6)
    t = np.sort(rng.uniform(0.2, 4, (6, 4)), axis=1)
    got = interval_depth(_t(mu), _t(sig), _t(om), _t(t)).numpy()
    for i in range(6):
        f = lambda s: om[i] * math.exp(-0.5 * ((s - mu[i]) / sig[i]) ** 2)
        for j in range(3):
            ref = integrate.quad(f, t[i, j], t[i, j + 1], epsabs=1e-14, epsrel=1e-12)[0]
            assert got[i, j] == pytest.approx(ref, rel=1e-10, abs=1e-14)


def test_penalty_vanishes_for_the_exact_optical_depth_and_is_the_square_sum_for_none():
    """With the exact optical depth of all particles on the ray, the gain over
    any interval is at least one particle's own depth there: P_i = 0. With a
    reconstruction that predicts no depth, P_i = sum_j tau_ij^2."""
    from oracle.quadrature import consistency_penalty, interval_depth
    rng = np.random.default_rng(22)
    n, tn = 7, 0.2
    mu, sig, om = rng.uniform(0.5, 3, n), rng.uniform(0.05, 0.6, n), rng.lognormal(0, 1, n)
    x = np.array([-1.15, -0.32, 0.32, 1.15])
    t = np.maximum(mu[:, None] + 3 * sig[:, None] * x[None, :], tn)

    def depth_all(tt):  # exact optical depth of the whole ray from t_n to tt
        return sum(om[k] * sig[k] * math.sqrt(math.pi / 2)
                   * (math.erf((tt - mu[k]) / (math.sqrt(2) * sig[k]))
                      - math.erf((tn - mu[k]) / (math.sqrt(2) * sig[k]))) for k in range(n))

    tau = np.array([[depth_all(v) for v in row] for row in t])
    p = consistency_penalty(_t(mu), _t(sig), _t(om), _t(tau), _t(t)).numpy()
    assert np.all(np.abs(p) < 1e-24)
    p0 = consistency_penalty(_t(mu), _t(sig), _t(om), _t(np.zeros_like(t)), _t(t)).numpy()
    tij = interval_depth(_t(mu), _t(sig), _t(om), _t(t)).numpy()
    assert np.allclose(p0, (tij ** 2).sum(1), rtol=1e-14)


def test_penalty_gradients_vs_central_differences():
    """Oracle autograd of a loss with a penalty term against central differences."""
    scene = _tiny_scene(5, 4)
    cam = W.camera_on_axis(2.0, 8, 8)
    opts = W.Options(n_moments=4, full_coverage=True)
    rng = np.random.default_rng(7)
    g_img = rng.normal(size=(64, 3))
    g_pen = rng.uniform(0.5, 1.5, 64)
    grads = oracle.render_backward(scene, cam, opts, g_img, grad_penalty=g_pen)
    r0 = oracle.render_image(scene, cam, opts)
    assert r0["penalty"].max() > 1e-6  # the penalty is active on this scene

    base = {k: np.asarray(getattr(scene, k), np.float64) for k in oracle.render.PARAMS}

    def loss64(params):
        sc = W.Scene(params["means"], params["scales"], params["quats"], params["densities"],
                     params["colors"], scene.sh_degree)
        r = oracle.render_image(sc, cam, opts)
        return float((r["image"] * g_img).sum() + (r["penalty"] * g_pen).sum())

    for name in ("means", "scales", "quats", "densities"):
        arr = base[name]
        for _ in range(3):
            idx = tuple(rng.integers(0, s) for s in arr.shape)
            h = 1e-6 * max(1.0, abs(arr[idx]))
            p = {k: v.copy() for k, v in base.items()}
            p[name][idx] += h
            lp = loss64(p)
            p[name][idx] -= 2 * h
            lm = loss64(p)
            fd = (lp - lm) / (2 * h)
            assert grads[name][idx] == pytest.approx(fd, rel=1e-5, abs=1e-8), name


def test_render_gradients_through_the_surrogate_vs_central_differences():
    """Oracle autograd of a render through the network (no rounding, so the
    loss is smooth) against central differences of the same render."""
    from oracle import surrogate as S
    scene = _tiny_scene(5, 4)
    cam = W.camera_on_axis(2.0, 8, 8)
    opts = W.Options(n_moments=6, full_coverage=True)
    theta = S.init_params(17)
    rng = np.random.default_rng(8)
    g_img = rng.normal(size=(64, 3))
    grads = oracle.render_backward(scene, cam, opts, g_img,
                                   tau_model=S.tau_model_torch(theta, network="exact"))
    base = {k: np.asarray(getattr(scene, k), np.float64) for k in oracle.render.PARAMS}
    model = S.tau_model(theta, bf16_mode=False)

    def loss64(params):
        sc = W.Scene(params["means"], params["scales"], params["quats"], params["densities"],
                     params["colors"], scene.sh_degree)
        return float((oracle.render_image(sc, cam, opts, tau_model=model)["image"] * g_img).sum())

    for name in ("means", "scales", "quats", "densities"):
        arr = base[name]
        for _ in range(3):
            idx = tuple(rng.integers(0, s) for s in arr.shape)
            h = 1e-6 * max(1.0, abs(arr[idx]))
            p = {k: v.copy() for k, v in base.items()}
            p[name][idx] += h
            lp = loss64(p)
            p[name][idx] -= 2 * h
            lm = loss64(p)
            fd = (lp - lm) / (2 * h)
            assert grads[name][idx] == pytest.approx(fd, rel=1e-5, abs=1e-8), name


# ---------------------------------------------------------------------------
# Adaptive density control (App. E): oracle.adc.
# ---------------------------------------------------------------------------

def test_split_constants_minimise_the_appendix_objective():
    """The printed (gamma, delta) sit at the minimum of the appendix's
    objective: minimising it from several starts lands within 0.01 of them,
    and their objective value is within 0.2% of the minimum. A plausible
    misreading (matching the densities without the transmittance) lands far
    from them."""
    from scipy import optimize
    from oracle import adc
    best = None
    for c0 in (1.0, 2.0, 3.0):
        for g0 in (0.5, 0.7, 0.9):
            r = optimize.minimize(lambda p: adc.split_objective(p[0], p[1]) if 0 < p[1] <= 1 else 1e9,
                                  [c0, g0], method="Nelder-Mead",
                                  options=dict(xatol=1e-9, fatol=1e-14, maxiter=4000))
            best = r if best is None or r.fun < best.fun else best
    c, g = best.x
    assert abs(g - adc.SPLIT_GAMMA) < 0.01
    assert abs(c * (1 - g) - adc.SPLIT_DELTA) < 0.01
    c_paper = adc.SPLIT_DELTA / (1 - adc.SPLIT_GAMMA)
    assert adc.split_objective(c_paper, adc.SPLIT_GAMMA) <= best.fun * 1.002
    # densities alone (no transmittance): a different optimum
    t = np.linspace(-12, 12, 24001)

    def dens_only(p):
        d = p[0] * (1 - p[1])
        r = np.exp(-0.5 * t * t) - np.exp(-(t - d) ** 2 / (2 * p[1] ** 2)) - np.exp(-(t + d) ** 2 / (2 * p[1] ** 2))
        return float((r * r).sum() * (t[1] - t[0]))
    r2 = optimize.minimize(dens_only, [1.5, 0.6], method="Nelder-Mead")
    assert abs(r2.x[1] - adc.SPLIT_GAMMA) > 0.1


def test_view_independent_opacity_is_the_opacity_along_the_shortest_axis():
    """1 - exp(-integral of the 3D density along the line through the centre
    in the direction of the smallest scale), integrated numerically."""
    from oracle import adc
    rng = np.random.default_rng(31)
    for _ in range(5):
        s = rng.uniform(0.05, 0.5, 3)
        q = rng.normal(size=4)
        w = rng.uniform(0.2, 5.0)
        mean = rng.normal(size=3)
        rot = quat_to_rot(torch.tensor(q)).numpy()
        prec = rot @ np.diag(1 / s ** 2) @ rot.T
        axis = rot[:, int(np.argmin(s))]

        def dens(t):
            x = mean + t * axis - mean
            return w * math.exp(-0.5 * x @ prec @ x)
        tau = integrate.quad(dens, -20 * s.max(), 20 * s.max(), epsabs=1e-14, epsrel=1e-12, limit=200)[0]
        assert adc.view_independent_opacity(s[None], np.array([w]))[0] == pytest.approx(1 - math.exp(-tau),
                                                                                        rel=1e-10)


def test_density_from_opacity_inverts_the_opacity_for_equal_scales():
    from oracle import adc
    s = np.full((4, 3), 0.2)
    o = np.array([0.01, 0.1, 0.5, 0.9])
    w = adc.density_from_opacity(o, s)
    assert np.allclose(adc.view_independent_opacity(s, w), o, rtol=1e-12)


def test_clone_keeps_the_density_field_and_split_follows_the_longest_axis():
    from oracle import adc
    rng = np.random.default_rng(5)
    n = 4
    means = rng.normal(size=(n, 3))
    scales = rng.uniform(0.05, 0.4, (n, 3))
    quats = rng.normal(size=(n, 4))
    dens = rng.uniform(0.5, 3, n)
    cols = rng.uniform(0, 1, (n, 3))
    action = np.array([adc.KEEP, adc.CLONE, adc.SPLIT, adc.PRUNE], np.int32)
    out = adc.apply(means, scales, quats, dens, cols, action)
    assert out["means"].shape == (5, 3)
    rot = quat_to_rot(torch.tensor(quats)).numpy()

    def field(m, s, r, w, x):
        d = x - m
        return w * math.exp(-0.5 * d @ (r @ np.diag(1 / s ** 2) @ r.T) @ d)
    for x in rng.normal(size=(6, 3)) * 0.3 + means[1]:
        both = sum(field(out["means"][k], out["scales"][k], rot[1], out["densities"][k], x) for k in (1, 2))
        assert both == pytest.approx(field(means[1], scales[1], rot[1], dens[1], x), rel=1e-12, abs=1e-300)
    k = int(np.argmax(scales[2]))
    a = rot[2][:, k]
    assert np.allclose(out["means"][3] + out["means"][4], 2 * means[2])
    assert np.allclose(out["means"][4] - out["means"][3], 2 * adc.SPLIT_DELTA * scales[2][k] * a)
    assert out["scales"][3][k] == pytest.approx(adc.SPLIT_GAMMA * scales[2][k])
    assert np.allclose(np.delete(out["scales"][3], k), np.delete(scales[2], k))


def test_plan_on_hand_built_particles():
    from oracle import adc
    scales = np.array([[0.01, 0.02, 0.03], [0.2, 0.2, 0.2], [0.2, 0.2, 0.2], [0.5, 0.2, 0.2], [0.2, 0.2, 0.2]])
    dens = np.array([0.1, 2.0, 2.0, 2.0, 2.0])   # the first is nearly transparent
    acc = np.array([[1, 1, 1], [0, 0, 0], [3e-4, 0, 0], [3e-4, 0, 0], [1e-5, 0, 0]], float)
    cnt = np.array([1, 0, 2, 2, 1])
    action, off, total = adc.plan(scales, dens, acc, cnt, min_opacity=0.005, grad_threshold=1e-4,
                                  split_scale=0.3)
    assert list(action) == [adc.PRUNE, adc.KEEP, adc.CLONE, adc.SPLIT, adc.KEEP]
    assert list(off) == [0, 0, 1, 3, 5] and total == 6


# ---------------------------------------------------------------------------
# The D-SSIM term of the objective: oracle.loss.
# ---------------------------------------------------------------------------

def test_ssim_against_a_brute_force_window_loop():
    """Every local statistic summed explicitly over the 11 x 11 window (zero
    outside the image) on a tiny image, against the separable version and the
    torch one."""
    from oracle import loss as Ls
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, (1, 9, 13, 3))
    y = np.clip(x + rng.normal(0, 0.1, x.shape), 0, 1)
    g = Ls.gaussian_window()
    w2 = np.outer(g, g)
    h, w = 9, 13
    ref = np.zeros((h, w, 3))
    for i in range(h):
        for j in range(w):
            acc = np.zeros((5, 3))
            for di in range(-5, 6):
                for dj in range(-5, 6):
                    ii, jj = i + di, j + dj
                    if 0 <= ii < h and 0 <= jj < w:
                        a, b = x[0, ii, jj], y[0, ii, jj]
                        acc += w2[di + 5, dj + 5] * np.stack([a, b, a * a, b * b, a * b])
            mx, my, ex, ey, exy = acc
            sx, sy, sxy = ex - mx * mx, ey - my * my, exy - mx * my
            ref[i, j] = ((2 * mx * my + Ls.C1) * (2 * sxy + Ls.C2)) / ((mx * mx + my * my + Ls.C1) * (sx + sy + Ls.C2))
    assert np.allclose(Ls.ssim_map(x, y)[0], ref, atol=1e-13)
    assert Ls.dssim_torch(torch.tensor(x), torch.tensor(y)).item() == pytest.approx(1 - ref.mean(), abs=1e-13)


def test_ssim_identity_symmetry_and_gradient():
    from oracle import loss as Ls
    rng = np.random.default_rng(4)
    x = rng.uniform(0, 1, (2, 16, 12, 3))
    y = rng.uniform(0, 1, x.shape)
    assert Ls.dssim(x, x) == pytest.approx(0.0, abs=1e-14)
    assert Ls.dssim(x, y) == pytest.approx(Ls.dssim(y, x), abs=1e-14)
    xt = torch.tensor(x, requires_grad=True)
    Ls.dssim_torch(xt, torch.tensor(y)).backward()
    gx = xt.grad.numpy()
    for _ in range(6):
        idx = tuple(int(rng.integers(0, s)) for s in x.shape)
        h = 1e-6
        xp = x.copy(); xp[idx] += h
        xm = x.copy(); xm[idx] -= h
        fd = (Ls.dssim(xp, y) - Ls.dssim(xm, y)) / (2 * h)
        assert gx[idx] == pytest.approx(fd, rel=1e-5, abs=1e-12)


# ---------------------------------------------------------------------------
# Trigonometric moments (Sec. 3.2, Eqs. 13-14, App. C) and bounds on the circle.
# ---------------------------------------------------------------------------

def test_trig_zeroth_moment_is_the_exact_optical_depth():
    from oracle.trig import particle_trig_moments
    rng = np.random.default_rng(21)
    mu, sig, om = _t(rng.uniform(-0.5, 6, 20)), _t(rng.uniform(0.02, 1.0, 20)), _t(rng.lognormal(0, 1, 20))
    tn = 0.2
    m = particle_trig_moments(mu, sig, om, tn, 3)
    for i in range(20):
        ref = integrate.quad(lambda t: om[i].item() * math.exp(-(t - mu[i].item()) ** 2 / (2 * sig[i].item() ** 2)),
                             tn, np.inf, epsabs=1e-13, epsrel=1e-11)[0]
        assert m[i, 0].real.item() == pytest.approx(ref, rel=1e-9, abs=1e-14)
        assert m[i, 0].imag.item() == 0.0


def test_trig_moment_closed_form_with_exact_erf_integrates_the_linearised_warp():
    """Eq. 14 with the complex erf evaluated exactly equals numerical
    integration of e^{i k (2 pi - theta)(G + G' (t - mu))} sigma(t) over
    [t_n, inf): the completion of the square and the t_f -> inf limit of the
    appendix's derivation."""
    from oracle.moments import warp, warp_prime
    from oracle.trig import THETA, particle_trig_moments
    rng = np.random.default_rng(22)
    tn = 0.2
    for _ in range(12):
        mu, sig, om = rng.uniform(-0.3, 5), rng.uniform(0.05, 1.5), rng.lognormal(0, 1)
        m = particle_trig_moments(_t([mu]), _t([sig]), _t([om]), tn, 3, exact_erf=True)[0]
        ms = max(mu, tn)
        gp = warp_prime(_t(ms), tn).item()
        g = warp(_t(ms), tn).item() + gp * (mu - ms)
        for k in range(4):
            a = k * (2 * math.pi - THETA)
            f = lambda t, part: om * math.exp(-(t - mu) ** 2 / (2 * sig * sig)) * part(a * (g + gp * (t - mu)))
            re = integrate.quad(lambda t: f(t, math.cos), tn, mu + 40 * sig + 1, limit=400, epsabs=1e-13)[0]
            im = integrate.quad(lambda t: f(t, math.sin), tn, mu + 40 * sig + 1, limit=400, epsabs=1e-13)[0]
            assert m[k].real.item() == pytest.approx(re, rel=1e-7, abs=1e-11)
            assert m[k].imag.item() == pytest.approx(im, rel=1e-7, abs=1e-11)


def test_trig_first_order_erf_error_is_second_order_and_local():
    """App. C's first-order expansion of erf in the imaginary direction: the
    error of 1 - erf(a - i b) shrinks at least as b^2 (halving b at least
    quarters it) and carries the factor e^{-a^2} (it fades away from the
    near bound)."""
    from scipy.special import erf as cerf
    for a in (-1.0, -0.3, 0.0, 0.4, 1.2):
        errs = []
        for b in (0.08, 0.04, 0.02):
            exact = 1 - cerf(a - 1j * b)
            approx = math.erfc(a) + 1j * b * 2 / math.sqrt(math.pi) * math.exp(-a * a)
            errs.append(abs(exact - approx))
        # at least second order (third where erf'' vanishes, at a = 0)
        assert errs[1] / errs[0] <= 0.27 and errs[2] / errs[1] <= 0.27
        # |second derivative of erf| = (4 / sqrt(pi)) |a| e^{-a^2}; the next term is b^3 order
        assert errs[0] <= 0.08 ** 2 / 2 * (4 / math.sqrt(math.pi)) * (abs(a) + 0.1) * math.exp(-a * a) + 1e-3


def _circle_measure(n_atoms, seed, arc=(0.0, 1.8 * math.pi)):
    rng = np.random.default_rng(seed)
    phi = np.sort(rng.uniform(*arc, n_atoms))
    while np.diff(phi).min() < 0.2:
        phi = np.sort(rng.uniform(*arc, n_atoms))
    w = rng.uniform(0.2, 1, n_atoms)
    return phi, w / w.sum()


def _trig_moments_of(phi, w, n):
    return np.array([(w * np.exp(1j * k * phi)).sum() for k in range(n + 1)])


@pytest.mark.parametrize("n", [2, 3])
def test_circle_canonical_representation_recovers_atomic_measure(n):
    """n + 1 atoms on the circle queried at one of them: the canonical
    representation is the measure itself (uniqueness of the Szego quadrature
    through a point)."""
    from oracle.trig import circle_canonical
    phi, w = _circle_measure(n + 1, 30 + n)
    c = torch.as_tensor(_trig_moments_of(phi, w, n))
    for j in range(n + 1):
        z, lam = circle_canonical(c[None], torch.as_tensor([np.exp(1j * phi[j])]), n)
        ang = np.mod(np.angle(z[0].numpy()), 2 * np.pi)
        order = np.argsort(ang)
        assert np.abs(ang[order] - phi).max() < 1e-9
        assert np.abs(lam[0].numpy()[order] - w).max() < 1e-9


@pytest.mark.parametrize("n", [2, 3])
def test_circle_nodes_on_the_circle_reproduce_the_moments(n):
    """For a measure with more than n + 1 atoms (positive definite Toeplitz
    matrix) the kernel polynomial's zeros lie on the unit circle and the
    atoms with their Christoffel weights reproduce c_0..c_n."""
    from oracle.trig import circle_canonical
    phi, w = _circle_measure(7, 40 + n)
    c = torch.as_tensor(_trig_moments_of(phi, w, n))
    for psi in (0.3, 2.0, 4.1, 5.5):
        z, lam = circle_canonical(c[None], torch.as_tensor([np.exp(1j * psi)]), n)
        zz, ll = z[0].numpy(), lam[0].numpy()
        assert np.abs(np.abs(zz) - 1).max() < 1e-10
        assert np.all(ll > 0)
        for k in range(n + 1):
            assert abs((ll * zz ** k).sum() - c[k].item()) < 1e-10



def test_cut_margin_is_the_distance_of_the_nearest_other_atom_to_the_cut():
    """The canonical representation through one atom of a three-atom measure
    (n = 2) is the measure itself, so the distance of the nearest other atom
    to the cut (angle 2 pi - theta / 2) is known in closed form; the query's
    own position does not count."""
    from oracle import trig as T
    cut = 2 * math.pi - 0.5 * T.THETA
    for d_cut, other, psi in [(0.01, 1.0, 3.0), (-0.02, 2.0, 4.0), (0.3, 2.5, cut + 1e-3)]:
        phis = np.array([cut + d_cut, other, psi])
        lam = np.array([0.3, 0.3, 0.4])
        c = torch.as_tensor([(lam * np.exp(1j * k * phis)).sum() for k in range(3)], dtype=torch.complex128)
        _, eps = T.uniform_mixture(c[None] / c[0], 2)
        assert float(eps[0]) == 0.0
        marg = T.cut_margin(c[None], torch.tensor([psi], dtype=torch.float64), 2)
        expect = min(abs(d_cut), abs(math.remainder(other - cut, 2 * math.pi)))
        assert abs(float(marg[0]) - expect) < 1e-9

@pytest.mark.parametrize("n", [2, 3])
def test_circle_query_weight_is_the_largest_point_mass(n):
    """U - L, the weight at the query, is the Christoffel number: the least
    integral of |p|^2 over polynomials of degree n with p(w) = 1 (solved as
    least squares on the measure's atoms) and the largest mass any measure on
    the circle with these moments can put at w (linear programming over a
    grid of the circle through w)."""
    from oracle.trig import circle_canonical
    phi, w = _circle_measure(9, 50 + n)
    c = _trig_moments_of(phi, w, n)
    for psi in (1.0, 3.3):
        z, lam = circle_canonical(torch.as_tensor(c)[None], torch.as_tensor([np.exp(1j * psi)]), n)
        v = np.exp(1j * np.outer(phi, np.arange(n + 1)))
        vw = np.exp(1j * psi * np.arange(n + 1))
        g = (v.conj().T * w) @ v
        a = np.linalg.solve(g, vw.conj())
        a /= vw @ a
        assert lam[0, 0].item() == pytest.approx(np.real(a.conj() @ g @ a), rel=1e-9)
        grid = np.mod(psi + np.linspace(0, 2 * math.pi, 2401)[:-1], 2 * math.pi)  # grid[0] = psi
        a_eq = np.vstack([np.cos(np.outer(np.arange(n + 1), grid)),
                          np.sin(np.outer(np.arange(1, n + 1), grid))])
        b_eq = np.concatenate([c.real, c.imag[1:]])
        obj = np.zeros(len(grid))
        obj[0] = -1.0
        lp = linprog(obj, A_eq=a_eq, b_eq=b_eq, bounds=(0, None), method="highs")
        assert lp.status == 0
        assert -lp.fun == pytest.approx(lam[0, 0].item(), rel=1e-3)


def test_circle_estimates_bracket_a_measure_whose_nodes_it_is():
    """With the query at one of n + 1 atoms of a depth measure, L and U are
    the measure's mass before the atom and through it (the estimate is exact
    there; the ordering starts at the wrapping zone)."""
    from oracle.trig import THETA, trig_bound_tau
    n = 3
    phi, w = _circle_measure(n + 1, 77, arc=(0.1, 2 * math.pi - THETA - 0.1))
    m = torch.as_tensor(1.3 * _trig_moments_of(phi, w, n))
    for j in range(n + 1):
        tau, lo, up = trig_bound_tau(m[None], _t([phi[j]]), n, 0.25)
        assert lo.item() == pytest.approx(w[:j].sum(), abs=1e-9)
        assert up.item() == pytest.approx(w[:j + 1].sum(), abs=1e-9)


def test_trig_single_colour_scene_renders_exact_opacity():
    """Eq. 15 with trigonometric moments: a single-colour scene renders
    c (1 - e^{-m_0}) + e^{-m_0} bg, whatever the reconstruction."""
    scene = _tiny_scene(4, 6, rgb=np.array([0.3, 0.6, 0.9]))
    cam = W.camera_on_axis(2.5, 24, 24)
    opts = W.Options(n_moments=4, basis="trigonometric")
    r = oracle.render_image(scene, cam, opts)
    m0 = r["moments"][:, 0]
    ok = r["opacity"] >= opts.eps
    expect = np.array([0.3, 0.6, 0.9])[None] * (1 - np.exp(-m0))[:, None]
    assert ok.sum() > 50
    assert np.allclose(r["image"][ok], expect[ok], atol=1e-12)


def test_tabulated_reconstruction_interpolates_and_converges():
    """The tabulated schedule (oracle.surrogate.tabulated): exact at the
    nodes, linear between them, and converging to the untabulated
    reconstruction as the nodes get denser (second order in their spacing)."""
    from oracle.surrogate import exact_model, tabulated
    rng = np.random.default_rng(90)
    grid = np.linspace(-3, 3, 2001)
    dens = sum(rng.uniform(0.2, 1) * np.exp(-(grid - rng.uniform(-2, 2)) ** 2 / rng.uniform(0.1, 0.5))
               for _ in range(4))
    mom = np.array([(dens * grid ** k).sum() for k in range(7)]) * 0.01
    b = mom / mom[0]
    mean, std = b[1], math.sqrt(b[2] - b[1] ** 2)
    base = exact_model(0.25, max_z=np.inf)
    y_nodes = mean + std * np.linspace(-4, 4, 32)
    tab = tabulated(base, 32, 4.0)
    q = lambda model, ys: model(torch.as_tensor(np.tile(mom, (len(ys), 1))), _t(ys)).numpy()
    assert np.abs(q(tab, y_nodes) - q(base, y_nodes)).max() < 1e-12
    mid = 0.5 * (y_nodes[:-1] + y_nodes[1:])
    assert np.abs(q(tab, mid) - 0.5 * (q(base, y_nodes[:-1]) + q(base, y_nodes[1:]))).max() < 1e-12
    ys = mean + std * rng.uniform(-3.5, 3.5, 400)
    errs = [np.abs(q(tabulated(base, g, 4.0), ys) - q(base, ys)).max() for g in (33, 65, 129)]
    assert errs[1] < 0.35 * errs[0] and errs[2] < 0.35 * errs[1]
