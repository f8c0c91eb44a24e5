"""The mODIL loss as a differentiable torch function.

The paper obtains the gradient of the discrete loss by automatic
differentiation (Sections 2.1, 2.2).  Here the gradient comes from the
library's hand-written adjoint kernels instead, wrapped in a
torch.autograd.Function so that the loss composes with torch code (other
loss terms, torch optimisers, schedulers).

Memory: the forward pass evaluates the loss only and saves nothing but the
parameter pack it was given; the backward pass recomputes the prolonged fine
field (Horner prolongation inside the fused kernels), the residuals and the
adjoint, and restricts the gradient to every level.  No fine field per level
is stored between the two passes.
"""
import torch

from .modil import Context


class ModilLoss(torch.autograd.Function):
    """loss = sum of all loss terms of all instances at the parameter pack theta."""

    @staticmethod
    def forward(ctx, theta, modil_ctx):
        terms = modil_ctx.loss(theta.detach())
        ctx.modil_ctx = modil_ctx
        ctx.save_for_backward(theta)
        return terms.sum()

    @staticmethod
    def backward(ctx, grad_out):
        (theta,) = ctx.saved_tensors
        _, grad = ctx.modil_ctx.loss_grad(theta.detach())
        return grad * grad_out.to(grad.dtype), None


def modil_loss(theta: torch.Tensor, modil_ctx: Context) -> torch.Tensor:
    """Differentiable total loss (FP64 scalar on the device) of the pack theta."""
    return ModilLoss.apply(theta, modil_ctx)
