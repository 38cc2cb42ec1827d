"""One training step of the paper's objective on the GPU, composed from the
library's entry points (argument marshalling only):

    L = (1 - ALPHA) L1 + ALPHA D-SSIM + LAMBDA L_consistency,

L_consistency the consistency penalty averaged over pixels. The render,
losses, adjoint, Adam updates and density-control statistics all run in the
library's kernels; torch provides the buffers."""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, Optional, Sequence

import torch

from . import loss as GL
from .adc import AdcState
from .render import Gaussians, Workspace, render_backward, render_forward
from .surrogate import adam_step

PARAMS = ("means", "scales", "quats", "densities", "colors")


@dataclass
class Adam:
    """Adam moments for the parameters given learning rates (others fixed)."""
    lrs: Dict[str, float]
    step: int = 0
    m: Dict[str, torch.Tensor] = field(default_factory=dict)
    v: Dict[str, torch.Tensor] = field(default_factory=dict)

    def update(self, g: Gaussians, grads: Dict[str, torch.Tensor]):
        self.step += 1
        for k, lr in self.lrs.items():
            p = getattr(g, k)
            if k not in self.m or self.m[k].shape != p.shape:
                self.m[k] = torch.zeros_like(p)
                self.v[k] = torch.zeros_like(p)
            adam_step(p, self.m[k], self.v[k], grads[k].contiguous(), self.step, lr)


def train_step(g: Gaussians, cams: Sequence, opts, target: torch.Tensor, adam: Adam,
               adc: Optional[AdcState] = None, ws: Optional[Workspace] = None,
               on_device: bool = False) -> Dict[str, torch.Tensor]:
    """Render, evaluate the objective, back-propagate, update g in place.
    Returns the loss terms as device scalars, and the render state under
    "state". With ``ws`` and ``on_device`` the step has no host round trip;
    ``state.check()`` then verifies that the frame fitted the workspace (a
    workspace sized before a densification step is replaced, or its capacity
    grows, after it)."""
    image, saved, state, pen = render_forward(g, cams, opts, ws=ws, penalty=True, on_device=on_device)
    l1, ds, gimg = GL.objective_image_grad(image, target)
    gpen = torch.full_like(pen, GL.LAMBDA / pen.numel())
    cons = GL.l1(pen, torch.zeros_like(pen))  # mean penalty (it is non-negative)
    grads = render_backward(g, cams, opts, state, saved, gimg, gpen)
    if adc is not None:
        adc.accumulate(grads["means"])
    adam.update(g, grads)
    total = (1 - GL.ALPHA) * l1 + GL.ALPHA * ds + GL.LAMBDA * cons
    return {"l1": l1, "dssim": ds, "consistency": cons, "total": total, "state": state}
