"""Adaptive density control of the density-based medium (App. E) through the
C ABI: view-independent opacity, initial densities, accumulation of the
absolute mean gradient, and one densify/prune step. Argument marshalling
only; every step runs in the library's kernels."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import torch

from . import _lib as L
from .render import Gaussians, _ptr, _stream

SPLIT_GAMMA = 0.6385502815246582
SPLIT_DELTA = 0.6128153090966912


def view_independent_opacity(g: Gaussians) -> torch.Tensor:
    out = torch.empty(g.n, dtype=torch.float32, device=g.means.device)
    L.check(L.load().mb_view_independent_opacity(ctypes.byref(g.struct()), _ptr(out), _stream()))
    return out


def density_from_opacity(opacity: torch.Tensor, scales: torch.Tensor) -> torch.Tensor:
    opacity = opacity.to(torch.float32).contiguous()
    scales = scales.to(torch.float32).contiguous()
    out = torch.empty(opacity.shape[0], dtype=torch.float32, device=opacity.device)
    L.check(L.load().mb_density_from_opacity(opacity.shape[0], _ptr(opacity), _ptr(scales), _ptr(out), _stream()))
    return out


@dataclass
class AdcState:
    """Accumulated absolute mean gradients [n,3] and counted views [n]."""
    grad_acc: torch.Tensor
    grad_count: torch.Tensor

    @staticmethod
    def zeros(n: int, device="cuda") -> "AdcState":
        return AdcState(torch.zeros(n, 3, dtype=torch.float32, device=device),
                        torch.zeros(n, dtype=torch.int32, device=device))

    def accumulate(self, g_means: torch.Tensor):
        g_means = g_means.to(torch.float32).contiguous()
        L.check(L.load().mb_adc_accumulate(g_means.shape[0], _ptr(g_means), _ptr(self.grad_acc),
                                           _ptr(self.grad_count), _stream()))


def plan(g: Gaussians, state: AdcState, min_opacity: float = 0.005, grad_threshold: float = 1e-4,
         split_scale: float = 0.01):
    """mb_adc_plan: (action [n] int32, offsets [n] int32, n_out) -- reads the
    new set's size back (one wait on the stream)."""
    lib = L.load()
    dev = g.means.device
    action = torch.empty(g.n, dtype=torch.int32, device=dev)
    offsets = torch.empty(g.n, dtype=torch.int32, device=dev)
    n_out = torch.empty(1, dtype=torch.int32, device=dev)
    ws = torch.empty(max(int(lib.mb_adc_workspace_bytes(g.n)), 256), dtype=torch.uint8, device=dev)
    p = L.MbAdcParams(min_opacity, grad_threshold, split_scale)
    L.check(lib.mb_adc_plan(ctypes.byref(g.struct()), _ptr(state.grad_acc), _ptr(state.grad_count),
                            ctypes.byref(p), _ptr(action), _ptr(offsets), _ptr(n_out), _ptr(ws), ws.numel(),
                            _stream()))
    return action, offsets, int(n_out.item())


def apply(g: Gaussians, action: torch.Tensor, offsets: torch.Tensor, n_out: int) -> Gaussians:
    """mb_adc_apply: the particle set after the step."""
    dev = g.means.device
    f = lambda *shape: torch.empty(*shape, dtype=torch.float32, device=dev)
    out = Gaussians(f(n_out, 3), f(n_out, 3), f(n_out, 4), f(n_out), f((n_out,) + tuple(g.colors.shape[1:])),
                    g.sh_degree)
    L.check(L.load().mb_adc_apply(ctypes.byref(g.struct()), _ptr(action), _ptr(offsets), _ptr(out.means),
                                  _ptr(out.scales), _ptr(out.quats), _ptr(out.densities), _ptr(out.colors),
                                  _stream()))
    return out


def densify_and_prune(g: Gaussians, state: AdcState, min_opacity: float = 0.005, grad_threshold: float = 1e-4,
                      split_scale: float = 0.01) -> Gaussians:
    action, offsets, n_out = plan(g, state, min_opacity, grad_threshold, split_scale)
    return apply(g, action, offsets, n_out)
