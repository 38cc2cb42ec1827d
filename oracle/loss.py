"""The D-SSIM term of the training objective (the Training and Densification
paragraph: L = (1 - alpha) L1 + alpha L_D-SSIM + lambda L_consistency with
alpha = 0.2, lambda = 0.1), float64.

TEST INFRASTRUCTURE: see the package docstring.

The paper extends the 3DGS losses and defers to that codebase for them, so
SSIM here is the structural similarity of Wang et al. as 3DGS evaluates it:
per colour channel, local means, variances and covariance under an 11 x 11
Gaussian window (sigma 1.5, normalised to sum 1, zero padding outside the
image), SSIM = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)
(s_x^2 + s_y^2 + C2)) with C1 = 0.01^2, C2 = 0.03^2, averaged over pixels and
channels; L_D-SSIM = 1 - SSIM.
"""
from __future__ import annotations

import numpy as np
from scipy.ndimage import correlate1d

WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2


def gaussian_window():
    x = np.arange(WINDOW) - WINDOW // 2
    g = np.exp(-x * x / (2 * SIGMA * SIGMA))
    return g / g.sum()


def _blur(img):
    """Separable window over the two image axes of [..., H, W, 3] arrays."""
    g = gaussian_window()
    out = correlate1d(img, g, axis=-3, mode="constant", cval=0.0)
    return correlate1d(out, g, axis=-2, mode="constant", cval=0.0)


def ssim_map(x, y):
    """Per-pixel, per-channel SSIM of images x, y [..., H, W, 3]."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mx, my = _blur(x), _blur(y)
    sxx = _blur(x * x) - mx * mx
    syy = _blur(y * y) - my * my
    sxy = _blur(x * y) - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def dssim(x, y):
    return float(1.0 - ssim_map(x, y).mean())


def dssim_torch(x, y):
    """The same loss in torch float64 (differentiable in x), images
    [C, H, W, 3]; the window as a 2D zero-padded correlation."""
    import torch
    import torch.nn.functional as F
    g = torch.as_tensor(gaussian_window(), dtype=torch.float64)
    w2 = (g[:, None] * g[None, :])[None, None]

    def blur(t):  # [C, H, W, 3] -> per channel plane
        c, h, w_, k = t.shape
        p = t.permute(0, 3, 1, 2).reshape(c * k, 1, h, w_)
        return F.conv2d(p, w2, padding=WINDOW // 2).reshape(c, k, h, w_).permute(0, 2, 3, 1)
    mx, my = blur(x), blur(y)
    sxx = blur(x * x) - mx * mx
    syy = blur(y * y) - my * my
    sxy = blur(x * y) - mx * my
    s = ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))
    return 1.0 - s.mean()
