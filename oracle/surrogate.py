"""Float64 reference of the learned surrogate of the reconstruction.

TEST INFRASTRUCTURE: see the package docstring. The surrogate is not part of
the paper, so nothing in the paper pins it ("parity unpinned" with respect to
the paper); this reference is pinned instead to central finite differences and
to torch float64 autograd of the same function.

Network: 7 inputs -> 64 -> 64 -> 1, tanh-GELU hidden layers, sigmoid output F
(the normalised optical depth at the query; tau = m_0 F); loss
mean_i (exp(-m0_i F_i) - t_i)^2. With ``bf16=True`` the reference reproduces
the rounding points of the bf16 kernels: weights (W1, W2, w3) and inputs
(split into a bf16 pair hi + lo), the hidden activation H1, and the
back-propagated dZ2 and dZ1 before they enter the matrix products.
Parameter order: W1[64][7], b1[64], W2[64][64] (out, in), b2[64], w3[64], b3.
"""
from __future__ import annotations

import numpy as np

H = 64
N_IN = 7
SIZES = {"W1": (H, N_IN), "b1": (H,), "W2": (H, H), "b2": (H,), "w3": (H,), "b3": (1,)}
N_PARAMS = sum(int(np.prod(s)) for s in SIZES.values())
GELU_C = 0.7978845608028654
GELU_A = 0.044715


def unpack(theta):
    out, o = {}, 0
    for k, s in SIZES.items():
        n = int(np.prod(s))
        out[k] = np.asarray(theta[o:o + n], np.float64).reshape(s)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[k], np.float64).reshape(-1) for k in SIZES])


def bf16(x):
    """Round to bfloat16 (nearest even) through float32."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(x):
    t = np.tanh(GELU_C * (x + GELU_A * x ** 3))
    return 0.5 * x * (1 + t)


def gelu_prime(x):
    t = np.tanh(GELU_C * (x + GELU_A * x ** 3))
    return 0.5 * (1 + t) + 0.5 * x * (1 - t * t) * GELU_C * (1 + 3 * GELU_A * x * x)


def init_params(seed: int = 0):
    """He-style initialisation (a reading: the optimiser setup is not given)."""
    rng = np.random.default_rng(seed)
    p = {"W1": rng.normal(0, np.sqrt(2.0 / N_IN), (H, N_IN)), "b1": np.zeros(H),
         "W2": rng.normal(0, np.sqrt(2.0 / H), (H, H)), "b2": np.zeros(H),
         "w3": rng.normal(0, np.sqrt(1.0 / H), H), "b3": np.zeros(1)}
    return pack(p)


def forward(theta, x, bf16_mode: bool = True):
    """x [n, 8] (6 features, query, m0): returns F [n] and the cache."""
    p = unpack(theta)
    r = bf16 if bf16_mode else (lambda v: np.asarray(v, np.float64))
    xin = np.asarray(x, np.float64)[:, :N_IN]
    if bf16_mode:
        hi = bf16(xin)
        lo = bf16(np.asarray(xin, np.float32).astype(np.float64) - hi)
        xq = hi + lo
    else:
        xq = xin
    w1, w2, w3 = r(p["W1"]), r(p["W2"]), r(p["w3"])
    z1 = xq @ w1.T + p["b1"]
    h1 = r(gelu(z1))
    z2 = h1 @ w2.T + p["b2"]
    a2 = gelu(z2)
    out = a2 @ w3 + p["b3"][0]
    f = 1.0 / (1.0 + np.exp(-out))
    return f, dict(xq=xq, xhi=hi if bf16_mode else xq, xlo=lo if bf16_mode else 0 * xq,
                   z1=z1, h1=h1, z2=z2, a2=a2, f=f, w1=w1, w2=w2, w3=w3)


def loss_grad(theta, x, t_target, bf16_mode: bool = True):
    """Loss mean (exp(-m0 F) - t)^2 and its gradient [P]."""
    x = np.asarray(x, np.float64)
    n = x.shape[0]
    f, c = forward(theta, x, bf16_mode)
    m0 = x[:, 7]
    tp = np.exp(-m0 * f)
    diff = tp - np.asarray(t_target, np.float64)
    loss = float(np.mean(diff * diff))
    r = bf16 if bf16_mode else (lambda v: np.asarray(v, np.float64))
    dout = 2.0 * diff / n * (-m0 * tp) * f * (1 - f)
    g = {}
    g["b3"] = np.array([dout.sum()])
    g["w3"] = c["a2"].T @ dout
    dz2 = dout[:, None] * c["w3"][None, :] * gelu_prime(c["z2"])
    g["b2"] = dz2.sum(0)
    dz2r = r(dz2)
    g["W2"] = dz2r.T @ c["h1"]
    dh1 = dz2r @ c["w2"]
    dz1 = dh1 * gelu_prime(c["z1"])
    g["b1"] = dz1.sum(0)
    dz1r = r(dz1)
    g["W1"] = dz1r.T @ c["xhi"] + dz1r.T @ c["xlo"]
    return loss, pack(g)


def adam(theta, m, v, grad, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
