"""Rotations, camera rays, the ray-space 1D Gaussian and SH colour (float64).

TEST INFRASTRUCTURE: see the package docstring.
"""
from __future__ import annotations

import math

import torch

DT = torch.float64


def quat_to_rot(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrix of the quaternion (w, x, y, z), normalised first.
    Sec. 3.1 parameterises the covariance as R S S^T R^T with R from a
    quaternion (the 3DGS parameterisation the paper defers to)."""
    q = q / q.norm(dim=-1, keepdim=True)
    w, x, y, z = q.unbind(-1)
    r = torch.stack([
        1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y),
    ], dim=-1)
    return r.reshape(q.shape[:-1] + (3, 3))


def camera_matrices(cam):
    """World-to-camera rotation, translation and the world-space origin."""
    w2c = torch.as_tensor(cam.world_to_cam, dtype=DT)
    r, t = w2c[:, :3], w2c[:, 3]
    origin = -(r.T @ t)
    return r, t, origin


def pixel_directions(cam, px: torch.Tensor, py: torch.Tensor) -> torch.Tensor:
    """Unit world-space ray directions through pixel centres.

    Sec. 3.3 maps a pixel p_hom = (u, v, 1) to d_p = normalize(K^-1 p_hom);
    pixel (x, y) has its centre at (x + 1/2, y + 1/2)."""
    r, _, _ = camera_matrices(cam)
    u = px.to(DT) + 0.5
    v = py.to(DT) + 0.5
    d_cam = torch.stack([(u - cam.cx) / cam.fx, (v - cam.cy) / cam.fy,
                         torch.ones_like(u)], dim=-1)
    d_cam = d_cam / d_cam.norm(dim=-1, keepdim=True)
    return d_cam @ r  # rows: R^T d_cam


def ray_gaussian(origin, d, mean, rot, scale, weight):
    """Eqs. 4-6 (App. A): the density of one Gaussian along the ray o + t d is
    omega * exp(-(t - mu)^2 / (2 Sigma^2)) with, for o_g = S^-1 R^T (o - mean)
    and d_g = S^-1 R^T d,
        Sigma^2 = 1 / (d_g . d_g),   mu = -(o_g . d_g) / (d_g . d_g),
        omega = w exp(K),  K = -1/2 o_g . o_g + 1/2 (o_g . d_g)^2 / (d_g . d_g).
    All arguments are batched over pairs; returns (mu, Sigma, omega)."""
    rt = rot.transpose(-1, -2)
    og = (rt @ (origin - mean).unsqueeze(-1)).squeeze(-1) / scale
    dg = (rt @ d.unsqueeze(-1)).squeeze(-1) / scale
    dd = (dg * dg).sum(-1)
    od = (og * dg).sum(-1)
    oo = (og * og).sum(-1)
    sigma2 = 1.0 / dd
    mu = -od / dd
    k = -0.5 * oo + 0.5 * od * od / dd
    omega = weight * torch.exp(k)
    return mu, torch.sqrt(sigma2), omega


# ---------------------------------------------------------------------------
# Spherical harmonics (emission colour, Sec. 3.1: degree <= 3, 48 coefficients).
# ---------------------------------------------------------------------------

def _double_factorial(k: int) -> int:
    out = 1
    while k > 1:
        out *= k
        k -= 2
    return out


def real_sh_basis(dirs: torch.Tensor, degree: int) -> torch.Tensor:
    """Real spherical harmonics Y_{l,m}, l <= degree, at unit directions.

    Built from the associated Legendre recursion (with the Condon-Shortley
    phase) and Re/Im of (x + i y)^m:
        Y_{l,0} = N_l0 P_l^0(z)
        Y_{l,m} = sqrt2 (-1)^m N_lm P_l^m(z)/sin^m(theta) Re((x+iy)^m),  m > 0
        Y_{l,-m}= sqrt2 (-1)^m N_lm P_l^m(z)/sin^m(theta) Im((x+iy)^m),  m > 0
    with N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).  Column l^2 + l + m."""
    x, y, z = dirs.unbind(-1)
    cols = [None] * ((degree + 1) ** 2)
    # Q_l^m(z) = P_l^m(z) / sin^m(theta) is a polynomial in z.
    re = [torch.ones_like(x)]
    im = [torch.zeros_like(x)]
    for m in range(1, degree + 1):
        r_prev, i_prev = re[-1], im[-1]
        re.append(r_prev * x - i_prev * y)
        im.append(r_prev * y + i_prev * x)
    for m in range(0, degree + 1):
        q_prev = None
        q = torch.full_like(z, float((-1) ** m * _double_factorial(2 * m - 1)))
        for l in range(m, degree + 1):
            if l == m + 1:
                q_prev, q = q, z * (2 * m + 1) * q
            elif l > m + 1:
                q_prev, q = q, ((2 * l - 1) * z * q - (l + m - 1) * q_prev) / (l - m)
            n_lm = math.sqrt((2 * l + 1) / (4 * math.pi)
                             * math.factorial(l - m) / math.factorial(l + m))
            if m == 0:
                cols[l * l + l] = n_lm * q
            else:
                s = math.sqrt(2.0) * (-1) ** m * n_lm
                cols[l * l + l + m] = s * q * re[m]
                cols[l * l + l - m] = s * q * im[m]
    return torch.stack(cols, dim=-1)


def sh_rgb(colors: torch.Tensor, sh_degree: int, means: torch.Tensor,
           origin: torch.Tensor) -> torch.Tensor:
    """Per-Gaussian RGB. With sh_degree < 0 the colours are RGB already;
    otherwise the SH expansion is evaluated at the per-Gaussian view direction
    normalize(mean - origin) and mapped as max(0, value + 1/2) (the 3DGS
    convention the paper defers to)."""
    if sh_degree < 0:
        return colors
    d = means - origin
    d = d / d.norm(dim=-1, keepdim=True)
    basis = real_sh_basis(d, sh_degree)  # [n, (d+1)^2]
    val = (basis.unsqueeze(-1) * colors).sum(-2)
    return torch.clamp_min(val + 0.5, 0.0)
