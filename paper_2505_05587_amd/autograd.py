"""PyTorch autograd over the HIP rasterizer, with the splitting matrix as a
side output of the backward pass (Sec. 4.4, Theorem 1).

forward  = project -> instance sort -> front-to-back blend (Eq. alpha_blend)
backward = blend backward + projection backward, which also accumulates
           S_i += sum_views sum_pixels dL/dalpha_i(x) * Hessian_p alpha_i(x)

For any scalar loss built from the returned image with torch operations, the
upstream gradient dL/dimage reaches the library unchanged (the fused L1 path
of the C ABI is the special case dL/dC = sign(C - target) / (3HW)).

State kept between forward and backward, per pixel: the final transmittance
and the index of the last blended entry (8 bytes), besides the projected
records and the instance list that the forward built.  Nothing is recomputed
in Python and nothing falls back to the CPU: every stage is a library kernel.
"""
from __future__ import annotations

import torch

from .pipeline import CameraBatch, Rasterizer


class SplatRenderer:
    """Owns the device buffers of one camera batch.  ``render(params, S)``
    returns the packed image [3 * total_pixels] (per view, planar RGB) as a
    tensor that is differentiable w.r.t. ``params`` [F, n]; its backward adds
    the splitting matrices into ``S`` [6, n] (entries xx xy xz yy yz zz) when
    one is given.

    One renderer serves one forward/backward pair at a time: a second forward
    before the first one's backward invalidates it (checked)."""

    def __init__(self, cams: CameraBatch, sh_degree: int, capacity: int = 0):
        self.ras = Rasterizer(cams, sh_degree, capacity)
        self.generation = 0

    @property
    def cams(self) -> CameraBatch:
        return self.ras.cams

    def render(self, params: torch.Tensor, S: torch.Tensor | None = None) -> torch.Tensor:
        return _RenderSplit.apply(params, self, S)

    def view_image(self, packed: torch.Tensor, v: int) -> torch.Tensor:
        return self.ras.cams.view_image(packed, v)


class _RenderSplit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, renderer: SplatRenderer, S):
        if params.dtype != torch.float32 or not params.is_cuda:
            raise TypeError("params must be a float32 CUDA tensor [F, n]")
        params = params.contiguous()
        ras = renderer.ras
        ras.forward(params)
        renderer.generation += 1
        ctx.renderer = renderer
        ctx.generation = renderer.generation
        ctx.S = S
        ctx.save_for_backward(params)
        return ras.image.clone()

    @staticmethod
    def backward(ctx, grad_image):
        renderer: SplatRenderer = ctx.renderer
        if renderer.generation != ctx.generation:
            raise RuntimeError("the renderer ran another forward before this backward")
        (params,) = ctx.saved_tensors
        ras = renderer.ras
        grads = torch.zeros_like(params)
        S = ctx.S
        if S is None:
            S = torch.zeros((6, params.shape[1]), dtype=torch.float32, device=params.device)
        elif S.shape != (6, params.shape[1]) or S.dtype != torch.float32 or not S.is_contiguous():
            raise ValueError("S must be a contiguous float32 tensor [6, n]")
        ras.backward(params, grads, S, dL_dimage=grad_image.contiguous().float())
        return grads, None, None


def l1_loss(renderer: SplatRenderer, packed: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    """Eq. (loss): sum over views of the per-view mean absolute error."""
    diff = (packed - target).abs()
    total = packed.new_zeros(())
    for v in range(renderer.cams.V):
        total = total + renderer.view_image(diff, v).mean()
    return total
