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

Inputs of the network at a query y of a pixel (``features``, ``query``): the
pixel's normalised moments b_1..b_6 in standardised form (the moments of the
measure after the increasing affine map y -> (y - mean) / std), each passed
through asinh, and the query mapped the same way, clamped to [-10, 10]. The
bounds of Sec. 3.2 are covariant under such maps (a reading stated with the
oracle's pixel basis), so the normalised optical depth at the query is a
function of these seven numbers alone; ``exact_model`` is that function and
pins the feature map (a render through it reproduces the plain render).
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


def input_grad(theta, x, bf16_mode: bool = True):
    """F [n] and dF/d(inputs) [n, 7] (6 features, query) by the chain rule
    through the network; with ``bf16_mode`` the back-propagated dZ2 and dZ1
    are rounded before their matrix products, as in ``loss_grad``."""
    f, c = forward(theta, x, bf16_mode)
    r = bf16 if bf16_mode else (lambda v: np.asarray(v, np.float64))
    dout = f * (1 - f)
    dz2 = dout[:, None] * c["w3"][None, :] * gelu_prime(c["z2"])
    dh1 = r(dz2) @ c["w2"]
    dz1 = dh1 * gelu_prime(c["z1"])
    return f, r(dz1) @ c["w1"]


def adam(theta, m, v, grad, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


MAX_Z = 10.0


def features(mom):
    """mom [P, 7] moments m_0..m_6 of a pixel in any increasing affine moment
    variable. Returns (feat [P, 6] = asinh of the standardised moments 1..6,
    mean [P], std [P]) of the normalised measure in that variable."""
    mom = np.asarray(mom, np.float64)
    b = mom / mom[:, :1]
    mean = b[:, 1]
    var = b[:, 2] - mean * mean
    std = np.sqrt(np.where(var > 0, var, 1.0))
    central = np.zeros((mom.shape[0], 7))
    for k in range(7):
        # E[(y - mean)^k] by the binomial theorem
        central[:, k] = sum(comb(k, j) * b[:, j] * (-mean) ** (k - j) for j in range(k + 1))
    std_mom = central[:, 1:] / std[:, None] ** np.arange(1, 7)[None, :]
    return np.arcsinh(std_mom), mean, std


def comb(k, j):
    from math import comb as _c
    return _c(k, j)


def query(y, mean, std, max_z: float = MAX_Z):
    """The query y in the standardised variable, clamped to [-max_z, max_z]."""
    return np.clip((np.asarray(y, np.float64) - mean) / std, -max_z, max_z)


def network_inputs(mom_q, y, max_z: float = MAX_Z):
    """Rows (6 features, query, m_0) for queries y [Q] of pixels with moments
    mom_q [Q, 7] (one row of moments per query)."""
    feat, mean, std = features(mom_q)
    z = query(y, mean, std, max_z)
    return np.concatenate([feat, z[:, None], np.asarray(mom_q, np.float64)[:, :1]], axis=1)


def tau_model(theta, bf16_mode: bool = True):
    """Optical depth m_0 F(inputs) of the network with parameters theta, in
    the (mom_q, y) -> tau form of the oracle renderer's reconstruction hook."""
    import torch

    def model(mom_q, y):
        m = mom_q.detach().numpy() if hasattr(mom_q, "detach") else np.asarray(mom_q)
        yy = y.detach().numpy() if hasattr(y, "detach") else np.asarray(y)
        x = network_inputs(m, yy)
        f, _ = forward(theta, x, bf16_mode)
        return torch.as_tensor(m[:, 0] * f, dtype=torch.float64)
    return model


def exact_model(beta: float, max_z: float = MAX_Z):
    """The target the network learns: the bound interpolation of Sec. 3.2
    evaluated from the network inputs alone (standardised moments recovered
    by sinh, m_0 = 1, query as given), times m_0. With max_z = inf it is the
    reconstruction itself, written in the network's inputs."""
    import torch
    from .bounds import bound_tau

    def model(mom_q, y):
        m = mom_q.detach().numpy() if hasattr(mom_q, "detach") else np.asarray(mom_q)
        yy = y.detach().numpy() if hasattr(y, "detach") else np.asarray(y)
        x = network_inputs(m, yy, max_z)
        b = np.concatenate([np.ones((x.shape[0], 1)), np.sinh(x[:, :6])], axis=1)
        tau, _, _ = bound_tau(torch.as_tensor(b), torch.as_tensor(x[:, 6]), 3, beta)
        return torch.as_tensor(m[:, 0]) * tau
    return model


def bounds_model(n_half: int, beta: float):
    """The moment bounds' interpolation of Sec. 3.2 (with the degenerate-
    measure rule) in the (mom_q, y) -> tau form, for any number of moments
    2 n_half: what the renderer uses when no model is given."""
    from .bounds import bound_tau

    def model(mom_q, y):
        tau, _, _ = bound_tau(mom_q, y, n_half, beta)
        return tau
    return model


TAB_NODES = 32
TAB_Z = 4.0


def tabulated(model, n_nodes: int = TAB_NODES, z_max: float = TAB_Z):
    """A reconstruction evaluated once per pixel at n_nodes equally spaced
    nodes z_g of the standardised query on [-z_max, z_max] (the table of the
    pixel) and linearly interpolated at each query's standardised position,
    clamped to the table's ends (an evaluation schedule, not in the paper:
    it applies to the plain bounds and to the learned surrogate alike). The
    nodes sit at y_g = mean + std z_g in the pixel's moment variable (mean and
    std of its normalised measure), so the table does not depend on that
    variable. ``model`` has the oracle renderer's (mom_q, y) -> tau form."""
    import torch
    zs = np.linspace(-z_max, z_max, n_nodes)

    def tab_model(mom_q, y):
        m = mom_q.detach().numpy() if hasattr(mom_q, "detach") else np.asarray(mom_q)
        yy = y.detach().numpy() if hasattr(y, "detach") else np.asarray(y)
        rows, inv = np.unique(m, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        m0 = np.where(rows[:, 0] > 0, rows[:, 0], 1.0)
        mean = rows[:, 1] / m0
        var = rows[:, 2] / m0 - mean * mean
        std = np.sqrt(np.where(var > 0, var, 1.0))
        node_y = mean[:, None] + std[:, None] * zs[None, :]
        tau = model(torch.as_tensor(np.repeat(rows, n_nodes, axis=0)),
                    torch.as_tensor(node_y.reshape(-1)))
        f = tau.detach().numpy().reshape(len(rows), n_nodes) / m0[:, None]
        z = np.clip((yy - mean[inv]) / std[inv], -z_max, z_max)
        u = (z + z_max) / (2 * z_max) * (n_nodes - 1)
        i0 = np.minimum(np.floor(u).astype(int), n_nodes - 2)
        fr = u - i0
        fq = (1 - fr) * f[inv, i0] + fr * f[inv, i0 + 1]
        return torch.as_tensor(m[:, 0] * fq, dtype=torch.float64)
    return tab_model


# ---------------------------------------------------------------------------
# Differentiable version (torch float64) for the gradient of a render through
# the surrogate. The bf16 rounding points of the kernels are kept in the
# forward values and passed straight through in the derivative (the kernels
# differentiate the network at its rounded values the same way).
# ---------------------------------------------------------------------------

def _bf16_t(x):
    import torch
    with torch.no_grad():
        r = torch.as_tensor(bf16(x.detach().numpy()), dtype=torch.float64)
    return x + (r - x).detach()


def forward_torch(theta, x):
    """F [n] of network inputs x [n, 7] (torch float64, differentiable in x);
    the same rounding points as `forward` with bf16_mode."""
    import torch
    p = {k: torch.as_tensor(v, dtype=torch.float64) for k, v in unpack(theta).items()}
    hi = _bf16_t(x)  # carries d/dx = 1
    lo = torch.as_tensor(bf16(x.detach().to(torch.float32).to(torch.float64).numpy() - hi.detach().numpy()),
                         dtype=torch.float64)
    xq = hi + lo
    w1, w2, w3 = (torch.as_tensor(bf16(p[k].numpy()), dtype=torch.float64) for k in ("W1", "W2", "w3"))
    z1 = xq @ w1.T + p["b1"]
    t1 = torch.tanh(GELU_C * (z1 + GELU_A * z1 ** 3))
    h1 = _bf16_t(0.5 * z1 * (1 + t1))
    z2 = h1 @ w2.T + p["b2"]
    t2 = torch.tanh(GELU_C * (z2 + GELU_A * z2 ** 3))
    a2 = 0.5 * z2 * (1 + t2)
    out = a2 @ w3 + p["b3"][0]
    return torch.sigmoid(out)


def _network_fn(theta, bf16_mode: bool):
    """F(x) as a torch function of x [n, 7] whose value is ``forward`` and
    whose derivative is ``input_grad`` (same rounding points)."""
    import torch

    class _Net(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x):
            f, dx = input_grad(theta, x.detach().numpy(), bf16_mode)
            ctx.save_for_backward(torch.as_tensor(dx, dtype=torch.float64))
            return torch.as_tensor(f, dtype=torch.float64)

        @staticmethod
        def backward(ctx, g):
            (dx,) = ctx.saved_tensors
            return g[:, None] * dx

    return _Net.apply


def tau_model_torch(theta, max_z: float = MAX_Z, network: str = "kernel"):
    """Differentiable optical depth m_0 F(inputs) through the network: the
    (mom_q, y) -> tau hook of the oracle renderer, for autograd. ``network``:
    "kernel" (bf16 rounding points of the kernels, forward and backward),
    "autograd" (``forward_torch``: rounded values, exact derivative) or
    "exact" (no rounding anywhere)."""
    import torch
    from math import comb as _c
    if network == "autograd":
        net = lambda x: forward_torch(theta, x)
    else:
        net = _network_fn(theta, network == "kernel")

    def model(mom_q, y):
        b = mom_q / mom_q[:, :1]
        mean = b[:, 1]
        var = b[:, 2] - mean * mean
        std = torch.sqrt(torch.where(var > 0, var, torch.ones_like(var)))
        cols = []
        for k in range(1, 7):
            ck = sum(_c(k, j) * b[:, j] * (-mean) ** (k - j) for j in range(k + 1))
            cols.append(torch.asinh(ck / std ** k))
        z = torch.clamp((y - mean) / std, -max_z, max_z)
        x = torch.stack(cols + [z], dim=1)
        return mom_q[:, 0] * net(x)
    return model
