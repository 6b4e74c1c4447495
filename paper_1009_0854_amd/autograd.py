"""torch.autograd.Function around the minimax RGB->CIELAB transform and its
hand-written backward (mact_transform / mact_transform_backward)."""
import torch

from . import _abi as A


class MactLab(torch.autograd.Function):
    """Linear float32 RGB (N, 3, H, W) -> CIELAB (N, 3, H, W), differentiable.

    Forward runs mact_transform (gamma none, CHW); backward runs
    mact_transform_backward, the chain rule through the same approximation."""

    @staticmethod
    def forward(ctx, x, params=None):
        from . import default_params, transform
        if x.dtype != torch.float32:
            raise TypeError("MactLab expects float32 linear RGB")
        p = params if params is not None else default_params(A.LAB)
        x = x.contiguous()
        ctx.save_for_backward(x)
        ctx.params = p
        return transform(x, params=p, layout="chw", gamma="none")

    @staticmethod
    def backward(ctx, grad_out):
        from . import transform_backward
        (x,) = ctx.saved_tensors
        g = transform_backward(x, grad_out.contiguous(), params=ctx.params, layout="chw")
        return g, None
