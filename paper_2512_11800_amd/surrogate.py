"""Learned surrogate of the moment -> optical-depth reconstruction.

Thin binding of the mb_mlp_* / mb_adam_step entry points (argument
marshalling only; every step runs in the library's kernels), plus the
training loop that drives them on harvested samples.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib as L
from .render import _ptr, _stream


def param_count() -> int:
    return int(L.load().mb_mlp_param_count())


def init_params(seed: int = 0, device="cuda") -> torch.Tensor:
    """He-style initial parameters (fp32 vector in the library's order)."""
    g = torch.Generator().manual_seed(seed)
    h, n_in = 64, 7
    parts = [torch.randn(h, n_in, generator=g, dtype=torch.float64) * (2.0 / n_in) ** 0.5,
             torch.zeros(h, dtype=torch.float64),
             torch.randn(h, h, generator=g, dtype=torch.float64) * (2.0 / h) ** 0.5,
             torch.zeros(h, dtype=torch.float64),
             torch.randn(h, generator=g, dtype=torch.float64) * (1.0 / h) ** 0.5,
             torch.zeros(1, dtype=torch.float64)]
    return torch.cat([p.reshape(-1) for p in parts]).to(torch.float32).to(device)


def mlp_pack(theta: torch.Tensor, packed: Optional[torch.Tensor] = None) -> torch.Tensor:
    lib = L.load()
    if packed is None:
        packed = torch.empty(int(lib.mb_mlp_packed_bytes()), dtype=torch.uint8, device=theta.device)
    L.check(lib.mb_mlp_pack(_ptr(theta), _ptr(packed), _stream()))
    return packed


def mlp_forward(packed: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    x = x.to(torch.float32).contiguous()
    out = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
    L.check(L.load().mb_mlp_forward(_ptr(packed), _ptr(x), x.shape[0], _ptr(out), _stream()))
    return out


class _Ws:
    buf: Optional[torch.Tensor] = None


def mlp_loss_grad(packed: torch.Tensor, x: torch.Tensor, t_target: torch.Tensor):
    """(loss [1], grad [P]) of mean (exp(-m0 F) - t)^2."""
    lib = L.load()
    x = x.to(torch.float32).contiguous()
    t_target = t_target.to(torch.float32).contiguous()
    n = x.shape[0]
    need = int(lib.mb_mlp_workspace_bytes(n))
    if _Ws.buf is None or _Ws.buf.numel() < need or _Ws.buf.device != x.device:
        _Ws.buf = torch.empty(need, dtype=torch.uint8, device=x.device)
    grad = torch.empty(param_count(), dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    L.check(lib.mb_mlp_loss_grad(_ptr(packed), _ptr(x), _ptr(t_target), n, _ptr(grad), _ptr(loss),
                                 _ptr(_Ws.buf), _Ws.buf.numel(), _stream()))
    return loss, grad


def adam_step(theta, m, v, grad, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    L.check(L.load().mb_adam_step(_ptr(theta), _ptr(m), _ptr(v), _ptr(grad), theta.numel(), int(step),
                                  float(lr), float(beta1), float(beta2), float(eps), _stream()))


def train(x: torch.Tensor, t: torch.Tensor, steps: int, batch: int = 65536, lr: float = 1e-3,
          seed: int = 0, theta: Optional[torch.Tensor] = None, log_every: int = 0,
          lr_final: Optional[float] = None):
    """Adam on minibatches drawn (seeded) from the harvested samples x [N, 8],
    t [N]; everything on the GPU. Returns (theta, packed weights, losses)."""
    device = x.device
    theta = init_params(seed, device) if theta is None else theta.clone()
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    gen = torch.Generator(device=device).manual_seed(seed)
    packed = mlp_pack(theta)
    losses = []
    n = x.shape[0]
    for step in range(1, steps + 1):
        idx = torch.randint(0, n, (batch,), device=device, generator=gen)
        loss, grad = mlp_loss_grad(packed, x[idx], t[idx])
        cur_lr = lr if lr_final is None else lr * (lr_final / lr) ** ((step - 1) / max(1, steps - 1))
        adam_step(theta, m, v, grad, step, cur_lr)
        mlp_pack(theta, packed)
        if log_every and (step % log_every == 0 or step == steps):
            losses.append((step, float(loss.item())))
    return theta, packed, losses


def _pairs_of(saved: torch.Tensor) -> int:
    """Covering (pixel, Gaussian) pairs of a forward render, from saved[..., 7]
    (the count n, or -(n + 1) where the Hankel factor took a bias)."""
    c = saved[..., 7]
    return int(torch.where(c < 0, -c - 1, c).sum().item())


def harvest(g, cams, opts, n_target: int, seed: int = 0, ws=None):
    """Training samples of the surrogate from the plain forward render of
    every camera in ``cams`` (one camera per call of
    mb_render_forward_harvest): about ``n_target`` queries drawn uniformly
    from all (pixel, covering Gaussian, quadrature edge) queries of the
    frames. The selection is a hash threshold, so the set is deterministic;
    the rows are returned in hash order, cut to the n_target smallest hashes.
    Returns (x [N, 8] = features, query, m_0; t [N] transmittance of the
    moment bounds; info dict)."""
    from .render import HARVEST_STRIDE, Workspace, render_forward_harvest
    cams = list(cams)
    dev = g.means.device
    ws = ws or Workspace(dev)
    nq = opts.n_intervals + 1
    # size the sampling rate from the first camera's query count
    probe = torch.empty(1, HARVEST_STRIDE, dtype=torch.float32, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    _, saved, _ = render_forward_harvest(g, cams[:1], opts, 0.0, seed, probe, count, ws)
    est = max(1, _pairs_of(saved) * nq * len(cams))
    rate = min(1.0, 1.2 * n_target / est)
    cap = int(1.5 * n_target) + 4096
    while True:
        samples = torch.empty(cap, HARVEST_STRIDE, dtype=torch.float32, device=dev)
        count.zero_()
        for i, cam in enumerate(cams):
            render_forward_harvest(g, [cam], opts, rate, (seed * 1000003 + i) & 0xFFFFFFFF,
                                     samples, count, ws)
        got = int(count.item())
        if got <= cap:
            break
        cap = int(got * 1.1) + 4096  # keep every selected sample: the set stays deterministic
    samples = samples[:got]
    key = samples[:, 9].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    order = torch.argsort(key * (1 << 31) + (samples[:, 10].view(torch.int32).to(torch.int64)))
    samples = samples[order[:n_target]]
    info = {"rate": rate, "selected": got, "queries_estimate": est, "kept": int(samples.shape[0])}
    return samples[:, :8].contiguous(), samples[:, 8].contiguous(), info
