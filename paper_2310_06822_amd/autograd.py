"""torch.autograd bridge for the asymmetric loss of Eq. 1.

    loss = BoundLoss.apply(theta, bound, q, y, alpha, beta)
    loss.backward()                 # theta.grad = dL/dtheta from the HIP kernel

The forward pass copies theta into the bound and runs the library's fused
forward / loss / backward kernel (nb_bound_loss_grad) once; the gradient it
produces is kept and scaled by the incoming gradient in backward, so no
activation crosses the C boundary.  Any torch optimiser can then step theta.
"""

from __future__ import annotations

import torch

from . import Bound, nb_bound_loss_grad, nb_bound_set_params


class BoundLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, bound: Bound, q: torch.Tensor, y: torch.Tensor, alpha: float,
                beta: float):
        theta_c = theta.detach().contiguous()
        nb_bound_set_params(bound.handle, theta_c)
        grad = torch.empty_like(theta_c)
        loss = torch.empty(1, dtype=torch.float32, device=theta.device)
        nb_bound_loss_grad(bound.handle, q, y, float(alpha), float(beta), grad, loss=loss)
        ctx.save_for_backward(grad)
        return loss[0]

    @staticmethod
    def backward(ctx, grad_out):
        (grad,) = ctx.saved_tensors
        return grad * grad_out, None, None, None, None, None


def bound_loss(theta: torch.Tensor, bound: Bound, q: torch.Tensor, y: torch.Tensor, alpha: float,
               beta: float = 1.0) -> torch.Tensor:
    return BoundLoss.apply(theta, bound, q, y, alpha, beta)
