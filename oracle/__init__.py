"""CPU oracle for moment-based order-independent 3D Gaussian splatting.

TEST INFRASTRUCTURE. This package is a plain, slow, float64 restatement of
the method (arXiv 2512.11800) used only to check the GPU path: only the tests,
``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg may import it.
The product path never calls into it and shares no code with it; the two meet
only in the seeded input generators of ``workloads``.

Each function follows the passage of the paper cited in its docstring:

* ``geometry``   -- rotation, camera rays, the ray-space 1D Gaussian (Eqs. 4-6,
                    App. A) and the SH emission colour (Sec. 3.1).
* ``proxy``      -- frustum culling and the confidence-interval screen proxy
                    (Sec. 3.3, Eqs. 16-21, App. D).
* ``moments``    -- the power-transform warp and the warped power moments
                    (Sec. 3.2, Eqs. 10-12, App. C).
* ``bounds``     -- moment-bound reconstruction of the optical depth through
                    the canonical representation (Sec. 3.2).
* ``quadrature`` -- sample spacing and the per-Gaussian quadrature (Eq. 7,
                    App. B) and opacity rescaling (Eq. 15).
* ``render``     -- the forward pass over a set of pixels and its gradient by
                    float64 autograd.
* ``exact``      -- the volume rendering equation (Eqs. 2-3) without the
                    moment approximation: the ground truth for image quality.
* ``surrogate``  -- float64 reference of the learned surrogate (not in the
                    paper) and the inputs it takes.

Where the paper is silent or garbled the oracle takes one reading; each one
is listed in the repository's design notes and named where it is used.
"""
from .geometry import quat_to_rot, pixel_directions, ray_gaussian, sh_rgb, real_sh_basis
from .moments import power_transform, warp, warp_prime, particle_moments
from .bounds import canonical_representation, bound_tau
from .quadrature import normal_quantiles, particle_quadrature, rescale
from .proxy import screen_proxy, covering_pairs
from .render import render_pixels, render_image, render_backward

__all__ = [
    "quat_to_rot", "pixel_directions", "ray_gaussian", "sh_rgb", "real_sh_basis",
    "power_transform", "warp", "warp_prime", "particle_moments",
    "canonical_representation", "bound_tau",
    "normal_quantiles", "particle_quadrature", "rescale",
    "screen_proxy", "covering_pairs",
    "render_pixels", "render_image", "render_backward",
]
