"""MI355X (gfx950) rendering path of moment-based order-independent 3D
Gaussian splatting (arXiv 2512.11800): HIP kernels behind the C ABI of
include/mb3dgs.h, with a thin ctypes binding and a torch.autograd wrapper."""
from ._lib import LIB_PATH, MbError, load
from .render import (HARVEST_STRIDE, Gaussians, RenderState, Workspace, camera_struct,
                     options_struct, project, render, render_backward, render_forward,
                     render_forward_harvest, render_forward_noalloc, render_forward_tabulated,
                     render_forward_surrogate, render_backward_surrogate, render_surrogate)

__all__ = ["LIB_PATH", "MbError", "load", "HARVEST_STRIDE", "Gaussians", "RenderState", "Workspace",
           "camera_struct", "options_struct", "project", "render", "render_backward",
           "render_forward", "render_forward_harvest", "render_forward_noalloc", "render_forward_tabulated",
           "render_forward_surrogate", "render_backward_surrogate", "render_surrogate"]
