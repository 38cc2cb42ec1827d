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


def options_struct(opts=None) -> L.MbOptions:
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
        basis = getattr(opts, "basis", "power")
        if basis not in ("power", "trigonometric"):
            raise ValueError(f"moment basis {basis!r}: 'power' or 'trigonometric'")
        o.basis = 1 if basis == "trigonometric" else 0
    return o


class Workspace:
    """Caller-owned device workspaces, grown on demand and reused."""

    def __init__(self, device="cuda"):
        self.device = torch.device(device)
        self.gws: Optional[torch.Tensor] = None
        self.pws: Optional[torch.Tensor] = None
        self.qws: Optional[torch.Tensor] = None
        self.tws: Optional[torch.Tensor] = None  # the tabulated schedule's per-pixel records and tables
        self.q_cap: int = 0
        self.capacity: int = 0  # list entries of renders with the count on the device

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
    q_cap: int = 0  # query capacity of a surrogate render
    n_gaussians: int = 0

    def entry_count(self) -> int:
        """The frame's list-entry total, read back from the device (waits)."""
        lib = L.load()
        n = ctypes.c_int64(0)
        gws = self.ws.gws
        L.check(lib.mb_entry_count(self.n_gaussians, self.n_cams, _ptr(gws), gws.numel(), ctypes.byref(n),
                                   _stream()))
        return int(n.value)

    def check(self):
        """For a render with the count on the device: raise when the frame had
        more list entries than its workspace holds (its image then misses
        them; render again after growing ``ws.capacity``)."""
        if self.n_entries != L.MB_ENTRIES_ON_DEVICE:
            return
        cap = int(L.load().mb_pair_capacity(self.ws.pws.numel(), self.n_cams, self.width, self.height))
        n = self.entry_count()
        if n > cap:
            self.ws.capacity = int(n * 1.25) + 4096
            raise RuntimeError(f"frame had {n} list entries, workspace holds {cap}; "
                               f"capacity raised to {self.ws.capacity}, render again")


def _cams(cams: Sequence) -> ctypes.Array:
    cams = list(cams)
    if not 1 <= len(cams) <= L.MB_MAX_CAMERAS:
        raise ValueError(f"1..{L.MB_MAX_CAMERAS} cameras supported")
    arr = (L.MbCamera * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = camera_struct(c)
    return arr


def project(g: Gaussians, cam, opts=None) -> torch.Tensor:
    """Screen proxies [n, 8] float64 (centre, major axis e1, half lengths, kept
    flag) via mb_project: the rectangles the coverage test uses."""
    lib = L.load()
    out = torch.empty(g.n, 8, dtype=torch.float64, device=g.means.device)
    L.check(lib.mb_project(ctypes.byref(g.struct()), ctypes.byref(camera_struct(cam)),
                           ctypes.byref(options_struct(opts)), _ptr(out), _stream()))
    return out


class _Frame:
    """Arguments of one forward call after mb_prepare (outputs allocated)."""

    def __init__(self, g: Gaussians, cams: Sequence, opts, ws: Optional[Workspace], on_device: bool = False):
        lib = L.load()
        self.cam_arr = _cams(cams)
        self.n_cams = len(self.cam_arr)
        self.n_gaussians = g.n
        self.width, self.height = int(self.cam_arr[0].width), int(self.cam_arr[0].height)
        self.o = options_struct(opts)
        self.gs = g.struct()
        self.ws = ws or Workspace(g.means.device)
        gws = self.ws._ensure("gws", lib.mb_gauss_workspace_bytes(g.n, self.n_cams))
        head = (ctypes.byref(self.gs), self.cam_arr, self.n_cams, ctypes.byref(self.o), _ptr(gws), gws.numel())
        if on_device and self.ws.capacity > 0:
            # the count stays on the device: no wait in this frame
            L.check(lib.mb_prepare(*head, None, _stream()))
            self.n_entries = L.MB_ENTRIES_ON_DEVICE
            need = self.ws.capacity
        else:
            n_entries = ctypes.c_int64(0)
            L.check(lib.mb_prepare(*head, ctypes.byref(n_entries), _stream()))
            self.n_entries = need = int(n_entries.value)
            if on_device:  # first frame: size the capacity from its count
                self.ws.capacity = need = int(need * 1.25) + 4096
                self.n_entries = L.MB_ENTRIES_ON_DEVICE
        self.ws._ensure("pws", lib.mb_pair_workspace_bytes(need, self.n_cams, self.width, self.height))
        dev = g.means.device
        self.image = torch.empty(self.n_cams, self.height, self.width, 3, dtype=torch.float32, device=dev)
        self.saved = torch.empty(self.n_cams, self.height, self.width, L.MB_SAVED_FLOATS_PER_PIXEL,
                                 dtype=torch.float32, device=dev)

    def head(self):
        """The arguments every forward entry point starts with."""
        ws = self.ws
        return (ctypes.byref(self.gs), self.cam_arr, self.n_cams, ctypes.byref(self.o), _ptr(ws.gws),
                ws.gws.numel(), _ptr(ws.pws), ws.pws.numel(), self.n_entries)

    def result(self):
        return self.image, self.saved, RenderState(self.ws, self.n_entries, self.n_cams, self.width,
                                                   self.height, n_gaussians=self.n_gaussians)


def render_forward(g: Gaussians, cams: Sequence, opts=None, ws: Optional[Workspace] = None,
                   penalty: bool = False, on_device: bool = False):
    """mb_prepare + mb_render_forward. Returns (image [C,H,W,3], saved [C,H,W,8],
    state), and the per-pixel consistency penalty [C,H,W] as a fourth item
    when ``penalty``. ``on_device`` keeps the list count on the device
    (MB_ENTRIES_ON_DEVICE) with the pair workspace sized for ``ws.capacity``
    (set from the first such frame's count): nothing waits, and
    ``state.check()`` verifies afterwards that the frame fitted."""
    f = _Frame(g, cams, opts, ws, on_device)
    pen = (torch.empty(f.n_cams, f.height, f.width, dtype=torch.float32, device=g.means.device)
           if penalty else None)
    L.check(L.load().mb_render_forward(*f.head(), _ptr(f.image), _ptr(f.saved), _ptr(pen), _stream()))
    return f.result() + ((pen,) if penalty else ())


def render_forward_noalloc(g: Gaussians, cams: Sequence, opts=None, image=None, saved=None):
    """mb_render_forward_noalloc: the forward render with the library's own
    device scratch in place of workspaces. ``image`` [C,H,W,3] and ``saved``
    [C,H,W,8] (float32, on the Gaussians' device) are allocated here unless
    given. Returns (image, saved, n_entries)."""
    lib = L.load()
    cam_arr = _cams(cams)
    n_cams = len(cam_arr)
    w, h = int(cam_arr[0].width), int(cam_arr[0].height)
    dev = g.means.device
    if image is None:
        image = torch.empty(n_cams, h, w, 3, dtype=torch.float32, device=dev)
    if saved is None:
        saved = torch.empty(n_cams, h, w, 8, dtype=torch.float32, device=dev)
    n_entries = ctypes.c_int64(0)
    gs = g.struct()
    o = options_struct(opts)
    L.check(lib.mb_render_forward_noalloc(ctypes.byref(gs), cam_arr, n_cams, ctypes.byref(o), _ptr(image),
                                          _ptr(saved), None, ctypes.byref(n_entries), _stream()))
    return image, saved, int(n_entries.value)


HARVEST_STRIDE = 12


def render_forward_harvest(g: Gaussians, cams: Sequence, opts, rate: float, seed: int,
                           samples: torch.Tensor, count: torch.Tensor,
                           ws: Optional[Workspace] = None):
    """mb_prepare + mb_render_forward_harvest: the plain forward render that
    also appends training samples of the surrogate to ``samples``
    [capacity, 12] (device float32) and advances ``count`` (device int32 [1]).
    Returns (image, saved, state)."""
    if samples.dtype != torch.float32 or samples.dim() != 2 or samples.shape[1] != HARVEST_STRIDE:
        raise ValueError("samples must be a float32 [capacity, 12] tensor")
    if count.dtype != torch.int32 or count.numel() != 1:
        raise ValueError("count must be a device int32 tensor of one element")
    f = _Frame(g, cams, opts, ws)
    L.check(L.load().mb_render_forward_harvest(*f.head(), float(rate), int(seed) & 0xFFFFFFFF,
                                               _ptr(samples), int(samples.shape[0]), _ptr(count),
                                               _ptr(f.image), _ptr(f.saved), _stream()))
    return f.result()


def render_forward_surrogate(g: Gaussians, cams: Sequence, opts, mlp_packed: torch.Tensor,
                             ws: Optional[Workspace] = None, query_capacity: Optional[int] = None,
                             check_capacity: bool = True, for_backward: bool = False):
    """mb_prepare + mb_render_forward_surrogate (the learned surrogate in place
    of the moment bounds). The query list lives in ``ws`` and is grown (and
    the frame rendered again) when a frame needs more queries than it holds;
    ``check_capacity=False`` skips that readback once ``ws`` is known to be
    large enough. ``for_backward`` sizes the query workspace for
    render_backward_surrogate. Returns (image, saved, state)."""
    lib = L.load()
    size_fn = lib.mb_query_workspace_bytes_backward if for_backward else lib.mb_query_workspace_bytes
    f = _Frame(g, cams, opts, ws)
    ws = f.ws
    if query_capacity is not None:
        ws.q_cap = max(ws.q_cap, int(query_capacity))
    if ws.q_cap == 0:
        ws.q_cap = 1 << 20
    while True:
        need = size_fn(f.n_cams, f.width, f.height, ws.q_cap)
        qws = ws._ensure("qws", need)
        L.check(lib.mb_render_forward_surrogate(*f.head(), _ptr(mlp_packed), _ptr(qws), qws.numel(),
                                                ws.q_cap, _ptr(f.image), _ptr(f.saved), _stream()))
        if not check_capacity:
            break
        n_q = int(qws[:8].view(torch.int64).item())
        if n_q <= ws.q_cap:
            break
        ws.q_cap = int(n_q * 1.1) + 1024
    img, saved, state = f.result()
    state.q_cap = ws.q_cap
    return img, saved, state


def render_forward_tabulated(g: Gaussians, cams: Sequence, opts, mlp_packed: Optional[torch.Tensor] = None,
                             n_nodes: int = 32, ws: Optional[Workspace] = None):
    """mb_prepare + mb_render_forward_tabulated: the reconstruction tabulated
    per pixel at ``n_nodes`` nodes of the standardised query and interpolated
    linearly; the moment bounds (``mlp_packed`` None) or the surrogate at the
    nodes. Returns (image, saved, state)."""
    lib = L.load()
    f = _Frame(g, cams, opts, ws)
    need = lib.mb_table_workspace_bytes(f.n_cams, f.width, f.height, int(n_nodes))
    tws = f.ws._ensure("tws", need)
    L.check(lib.mb_render_forward_tabulated(*f.head(), _ptr(mlp_packed), int(n_nodes), _ptr(tws), tws.numel(),
                                            _ptr(f.image), _ptr(f.saved), _stream()))
    return f.result()


def _grad_outputs(g: Gaussians):
    return {k: torch.empty_like(getattr(g, k)) for k in ("means", "scales", "quats", "densities", "colors")}


def render_backward_surrogate(g: Gaussians, cams: Sequence, opts, state: RenderState, saved: torch.Tensor,
                              grad_image: torch.Tensor, mlp_packed: torch.Tensor):
    """mb_render_backward_surrogate after render_forward_surrogate(...,
    for_backward=True) with the same weights. Returns a dict of gradients
    shaped like the inputs."""
    lib = L.load()
    cam_arr = _cams(cams)
    o = options_struct(opts)
    grad_image = grad_image.to(torch.float32).contiguous()
    out = _grad_outputs(g)
    ws = state.ws
    L.check(lib.mb_render_backward_surrogate(
        ctypes.byref(g.struct()), cam_arr, len(cam_arr), ctypes.byref(o), _ptr(ws.gws), ws.gws.numel(),
        _ptr(ws.pws), ws.pws.numel(), state.n_entries, _ptr(mlp_packed), _ptr(ws.qws), ws.qws.numel(),
        state.q_cap, _ptr(saved), _ptr(grad_image), _ptr(out["means"]), _ptr(out["scales"]),
        _ptr(out["quats"]), _ptr(out["densities"]), _ptr(out["colors"]), _stream()))
    return out


def render_backward(g: Gaussians, cams: Sequence, opts, state: RenderState, saved: torch.Tensor,
                    grad_image: torch.Tensor, grad_penalty: Optional[torch.Tensor] = None):
    """mb_render_backward. Returns a dict of gradients shaped like the inputs.
    ``grad_penalty`` [C,H,W] adds the gradient of a loss term on the
    consistency penalty."""
    lib = L.load()
    cam_arr = _cams(cams)
    o = options_struct(opts)
    grad_image = grad_image.to(torch.float32).contiguous()
    if grad_penalty is not None:
        grad_penalty = grad_penalty.to(torch.float32).contiguous()
    out = _grad_outputs(g)
    ws = state.ws
    L.check(lib.mb_render_backward(ctypes.byref(g.struct()), cam_arr, len(cam_arr), ctypes.byref(o),
                                   _ptr(ws.gws), ws.gws.numel(), _ptr(ws.pws), ws.pws.numel(),
                                   state.n_entries, _ptr(saved), _ptr(grad_image), _ptr(grad_penalty),
                                   _ptr(out["means"]), _ptr(out["scales"]), _ptr(out["quats"]),
                                   _ptr(out["densities"]), _ptr(out["colors"]), _stream()))
    return out


class _MomentRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, scales, quats, densities, colors, sh_degree, cams, opts, with_penalty):
        g = Gaussians(means.contiguous(), scales.contiguous(), quats.contiguous(),
                      densities.contiguous(), colors.contiguous(), sh_degree)
        out = render_forward(g, cams, opts, penalty=with_penalty)
        image, saved, state = out[:3]
        ctx.g, ctx.cams, ctx.opts, ctx.state = g, cams, opts, state
        ctx.with_penalty = with_penalty
        ctx.save_for_backward(saved)
        return (image, out[3]) if with_penalty else image

    @staticmethod
    def backward(ctx, grad_image, grad_penalty=None):
        (saved,) = ctx.saved_tensors
        if grad_image is None:
            grad_image = torch.zeros(ctx.state.n_cams, ctx.state.height, ctx.state.width, 3,
                                     dtype=torch.float32, device=saved.device)
        grads = render_backward(ctx.g, ctx.cams, ctx.opts, ctx.state, saved, grad_image,
                                grad_penalty if ctx.with_penalty else None)
        return (grads["means"], grads["scales"], grads["quats"], grads["densities"],
                grads["colors"], None, None, None, None)


def render(means, scales, quats, densities, colors, cams, opts=None, sh_degree: int = -1,
           with_penalty: bool = False):
    """Differentiable render [C,H,W,3] of the Gaussians from ``cams``; with
    ``with_penalty`` also the per-pixel consistency penalty [C,H,W] (App. E),
    so a loss can add lambda * mean(penalty)."""
    return _MomentRender.apply(means, scales, quats, densities, colors, sh_degree, list(cams), opts,
                               with_penalty)


class _SurrogateRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, scales, quats, densities, colors, sh_degree, cams, opts, mlp_packed, ws):
        g = Gaussians(means.contiguous(), scales.contiguous(), quats.contiguous(),
                      densities.contiguous(), colors.contiguous(), sh_degree)
        image, saved, state = render_forward_surrogate(g, cams, opts, mlp_packed, ws=ws, for_backward=True)
        ctx.g, ctx.cams, ctx.opts, ctx.state, ctx.packed = g, cams, opts, state, mlp_packed
        ctx.save_for_backward(saved)
        return image

    @staticmethod
    def backward(ctx, grad_image):
        (saved,) = ctx.saved_tensors
        grads = render_backward_surrogate(ctx.g, ctx.cams, ctx.opts, ctx.state, saved, grad_image, ctx.packed)
        return (grads["means"], grads["scales"], grads["quats"], grads["densities"],
                grads["colors"], None, None, None, None, None)


def render_surrogate(means, scales, quats, densities, colors, cams, mlp_packed: torch.Tensor, opts=None,
                     sh_degree: int = -1, ws: Optional[Workspace] = None):
    """Differentiable render [C,H,W,3] through the learned surrogate (weights
    ``mlp_packed`` from surrogate.mlp_pack, held fixed: they are trained from
    harvested samples, not through the image). ``ws`` keeps the query list
    between the forward and backward calls; a fresh one is made when None."""
    return _SurrogateRender.apply(means, scales, quats, densities, colors, sh_degree, list(cams), opts,
                                  mlp_packed, ws or Workspace(means.device))
