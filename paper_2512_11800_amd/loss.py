"""The D-SSIM term of the training objective through the C ABI (mb_dssim),
and a torch.autograd.Function around it. Argument marshalling only. The
paper weighs it as (1 - ALPHA) L1 + ALPHA D-SSIM + LAMBDA L_consistency."""
from __future__ import annotations

from typing import Optional

import torch

from . import _lib as L
from .render import _ptr, _stream

ALPHA = 0.2    # weight of D-SSIM against L1
LAMBDA = 0.1   # weight of the consistency penalty


def dssim(image: torch.Tensor, target: torch.Tensor, grad: Optional[torch.Tensor] = None,
          grad_scale: float = 1.0) -> torch.Tensor:
    """1 - mean SSIM of image against target ([C,H,W,3]); when ``grad`` is
    given, grad_scale * d loss / d image is added to it. Returns the loss as a
    device scalar."""
    lib = L.load()
    image = image.to(torch.float32).contiguous()
    target = target.to(torch.float32).contiguous()
    c, h, w, _ = image.shape
    loss = torch.empty(1, dtype=torch.float32, device=image.device)
    ws = torch.empty(max(int(lib.mb_dssim_workspace_bytes(c, w, h)), 256), dtype=torch.uint8,
                     device=image.device)
    L.check(lib.mb_dssim(_ptr(image), _ptr(target), c, w, h, float(grad_scale), _ptr(loss), _ptr(grad), _ptr(ws),
                         ws.numel(), _stream()))
    return loss[0]


def l1(image: torch.Tensor, target: torch.Tensor, grad: Optional[torch.Tensor] = None,
       grad_scale: float = 1.0) -> torch.Tensor:
    """mean |image - target|; when ``grad`` is given, grad_scale d loss / d
    image is added to it. Returns the loss as a device scalar."""
    lib = L.load()
    image = image.to(torch.float32).contiguous()
    target = target.to(torch.float32).contiguous()
    loss = torch.empty(1, dtype=torch.float32, device=image.device)
    ws = torch.empty(int(lib.mb_l1_workspace_bytes()), dtype=torch.uint8, device=image.device)
    L.check(lib.mb_l1(_ptr(image), _ptr(target), image.numel(), float(grad_scale), _ptr(loss), _ptr(grad),
                      _ptr(ws), ws.numel(), _stream()))
    return loss[0]


def objective_image_grad(image: torch.Tensor, target: torch.Tensor):
    """(1 - ALPHA) L1 + ALPHA D-SSIM of the image: returns (l1, dssim, grad)
    with grad = d/d image of the weighted sum, both terms' kernels adding
    into one buffer."""
    grad = torch.zeros_like(image, dtype=torch.float32).contiguous()
    a = l1(image, target, grad, 1.0 - ALPHA)
    b = dssim(image, target, grad, ALPHA)
    return a, b, grad


class DSsim(torch.autograd.Function):
    """D-SSIM(image, target), differentiable in image."""

    @staticmethod
    def forward(ctx, image, target):
        ctx.save_for_backward(image, target)
        return dssim(image, target)

    @staticmethod
    def backward(ctx, g):
        image, target = ctx.saved_tensors
        grad = torch.zeros_like(image, dtype=torch.float32).contiguous()
        dssim(image, target, grad, 1.0)
        return grad * g, None
