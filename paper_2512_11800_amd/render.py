"""Python face of the HIP rendering path.

``render_forward`` / ``render_backward`` have the names and arguments of the
C entry points (include/mb3dgs.h); torch supplies device memory (caller-side
workspaces grown on demand) and the current stream. ``render`` wraps both in
a torch.autograd.Function. Every step of the path runs in the library's
kernels; this module only marshals arguments.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch

from . import _lib as L


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _f32(t, device) -> torch.Tensor:
    return torch.as_tensor(t, dtype=torch.float32, device=device).contiguous()


@dataclass
class Gaussians:
    """Device tensors of a Gaussian set (float32, contiguous)."""
    means: torch.Tensor
    scales: torch.Tensor
    quats: torch.Tensor
    densities: torch.Tensor
    colors: torch.Tensor
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @staticmethod
    def from_scene(scene, device="cuda") -> "Gaussians":
        return Gaussians(_f32(scene.means, device), _f32(scene.scales, device),
                         _f32(scene.quats, device), _f32(scene.densities, device),
                         _f32(scene.colors, device), int(scene.sh_degree))

    def struct(self) -> L.MbGaussians:
        for t in (self.means, self.scales, self.quats, self.densities, self.colors):
            if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError("Gaussian tensors must be contiguous float32 CUDA tensors")
        return L.MbGaussians(self.n, self.sh_degree, _ptr(self.means), _ptr(self.scales),
                             _ptr(self.quats), _ptr(self.densities), _ptr(self.colors))


def camera_struct(cam) -> L.MbCamera:
    c = L.MbCamera()
    w2c = [float(v) for v in torch.as_tensor(cam.world_to_cam, dtype=torch.float64).reshape(-1)]
    c.world_to_cam = (ctypes.c_float * 12)(*w2c)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    c.t_near = float(cam.t_near)
    c.background = (ctypes.c_float * 3)(*[float(v) for v in cam.background])
    return c


def options_struct(opts=None, surrogate: Optional[torch.Tensor] = None) -> L.MbOptions:
    o = L.MbOptions()
    L.load().mb_default_options(ctypes.byref(o))
    if opts is not None:
        o.n_moments = int(opts.n_moments)
        o.n_intervals = int(opts.n_intervals)
        o.kappa = float(opts.kappa)
        o.conf_c = float(opts.conf_c)
        o.beta = float(opts.beta)
        o.eps = float(opts.eps)
        o.full_coverage = int(bool(getattr(opts, "full_coverage", False)))
        o.recon = int(getattr(opts, "recon", 0))
    if surrogate is not None:
        o.surrogate = surrogate.data_ptr()
    return o


class Workspace:
    """Caller-owned device workspaces, grown on demand and reused."""

    def __init__(self, device="cuda"):
        self.device = torch.device(device)
        self.gws: Optional[torch.Tensor] = None
        self.pws: Optional[torch.Tensor] = None

    def _ensure(self, name: str, nbytes: int) -> torch.Tensor:
        cur = getattr(self, name)
        if cur is None or cur.numel() < nbytes:
            cur = torch.empty(max(int(nbytes * 1.25), 256), dtype=torch.uint8, device=self.device)
            setattr(self, name, cur)
        return cur


@dataclass
class RenderState:
    """What a forward render leaves for its backward pass."""
    ws: Workspace
    n_entries: int
    n_cams: int
    width: int
    height: int


def _cams(cams: Sequence) -> ctypes.Array:
    cams = list(cams)
    if not 1 <= len(cams) <= L.MB_MAX_CAMERAS:
        raise ValueError(f"1..{L.MB_MAX_CAMERAS} cameras supported")
    arr = (L.MbCamera * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = camera_struct(c)
    return arr


def project(g: Gaussians, cam, opts=None) -> torch.Tensor:
    """Screen proxies [n, 8] (centre, e1, half lengths, kept flag) via mb_project."""
    lib = L.load()
    out = torch.empty(g.n, 8, dtype=torch.float32, device=g.means.device)
    L.check(lib.mb_project(ctypes.byref(g.struct()), ctypes.byref(camera_struct(cam)),
                           ctypes.byref(options_struct(opts)), _ptr(out), _stream()))
    return out


def render_forward(g: Gaussians, cams: Sequence, opts=None, ws: Optional[Workspace] = None,
                   surrogate: Optional[torch.Tensor] = None):
    """mb_prepare + mb_render_forward. Returns (image [C,H,W,3], saved [C,H,W,8], state)."""
    lib = L.load()
    cam_arr = _cams(cams)
    n_cams = len(cam_arr)
    width, height = int(cam_arr[0].width), int(cam_arr[0].height)
    o = options_struct(opts, surrogate)
    gs = g.struct()
    ws = ws or Workspace(g.means.device)
    gbytes = lib.mb_gauss_workspace_bytes(g.n, n_cams)
    gws = ws._ensure("gws", gbytes)
    n_entries = ctypes.c_int64(0)
    L.check(lib.mb_prepare(ctypes.byref(gs), cam_arr, n_cams, ctypes.byref(o), _ptr(gws),
                           gws.numel(), ctypes.byref(n_entries), _stream()))
    pbytes = lib.mb_pair_workspace_bytes(n_entries.value, n_cams, width, height)
    pws = ws._ensure("pws", pbytes)
    image = torch.empty(n_cams, height, width, 3, dtype=torch.float32, device=g.means.device)
    saved = torch.empty(n_cams, height, width, L.MB_SAVED_FLOATS_PER_PIXEL, dtype=torch.float32,
                        device=g.means.device)
    L.check(lib.mb_render_forward(ctypes.byref(gs), cam_arr, n_cams, ctypes.byref(o), _ptr(gws),
                                  gws.numel(), _ptr(pws), pws.numel(), n_entries.value,
                                  _ptr(image), _ptr(saved), _stream()))
    return image, saved, RenderState(ws, int(n_entries.value), n_cams, width, height)


def render_backward(g: Gaussians, cams: Sequence, opts, state: RenderState, saved: torch.Tensor,
                    grad_image: torch.Tensor, surrogate: Optional[torch.Tensor] = None):
    """mb_render_backward. Returns a dict of gradients shaped like the inputs."""
    lib = L.load()
    cam_arr = _cams(cams)
    o = options_struct(opts, surrogate)
    grad_image = grad_image.to(torch.float32).contiguous()
    out = {k: torch.empty_like(getattr(g, k)) for k in ("means", "scales", "quats", "densities", "colors")}
    ws = state.ws
    L.check(lib.mb_render_backward(ctypes.byref(g.struct()), cam_arr, len(cam_arr), ctypes.byref(o),
                                   _ptr(ws.gws), ws.gws.numel(), _ptr(ws.pws), ws.pws.numel(),
                                   state.n_entries, _ptr(saved), _ptr(grad_image),
                                   _ptr(out["means"]), _ptr(out["scales"]), _ptr(out["quats"]),
                                   _ptr(out["densities"]), _ptr(out["colors"]), _stream()))
    return out


class _MomentRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, scales, quats, densities, colors, sh_degree, cams, opts, surrogate):
        g = Gaussians(means.contiguous(), scales.contiguous(), quats.contiguous(),
                      densities.contiguous(), colors.contiguous(), sh_degree)
        image, saved, state = render_forward(g, cams, opts, surrogate=surrogate)
        ctx.g, ctx.cams, ctx.opts, ctx.state, ctx.surrogate = g, cams, opts, state, surrogate
        ctx.save_for_backward(saved)
        return image

    @staticmethod
    def backward(ctx, grad_image):
        (saved,) = ctx.saved_tensors
        grads = render_backward(ctx.g, ctx.cams, ctx.opts, ctx.state, saved, grad_image,
                                surrogate=ctx.surrogate)
        return (grads["means"], grads["scales"], grads["quats"], grads["densities"],
                grads["colors"], None, None, None, None)


def render(means, scales, quats, densities, colors, cams, opts=None, sh_degree: int = -1,
           surrogate: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Differentiable render [C,H,W,3] of the Gaussians from ``cams``."""
    return _MomentRender.apply(means, scales, quats, densities, colors, sh_degree, list(cams),
                               opts, surrogate)
