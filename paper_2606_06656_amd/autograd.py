"""The FE objective as a differentiable torch operation.

`FEObjective.apply(x, problem)` maps restart rows x (R, n) float32 on the GPU to
F(x) (R,) = sum_c w_c FE_c(x_r) (Background, "Satisfaction as Optimisation").
The forward pass runs the library's evaluation kernel, which produces the
gradient in the same pass; backward returns grad_F[:, None] * dF/dx.

The relaxation is defined on the cube Q^n = [-1, 1]^n, and the library's exact
fixed-point accumulation is scaled for it: every objective and gradient term is
bounded by its constraint's weight there, but outside the cube the products
prod_i (1 +- x_i)/2 grow geometrically with the constraint length and the
fixed-point sums would overflow.  forward() therefore rejects any entry with
|x| > 1 (or NaN) with a ValueError instead of returning a wrong value.
"""
from __future__ import annotations

import torch

from . import pcls


class FEObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, problem: "pcls.Problem"):
        if x.dim() != 2 or x.shape[1] != problem.n:
            raise ValueError(f"x must be (R, {problem.n}), got {tuple(x.shape)}")
        if x.device != problem.device:
            raise ValueError("x must live on the problem's device")
        if not bool(torch.all(x.detach().abs() <= 1)):
            raise ValueError("x must lie in [-1, 1]^n (the cube the objective and its fixed-point scales are "
                             "defined on)")
        R = x.shape[0]
        X = problem.new_state(R)
        X[:, :R] = x.detach().to(torch.float32).T
        obj, grad = problem.evaluate(X, R, want_grad=ctx.needs_input_grad[0])
        if grad is not None:
            ctx.save_for_backward(grad[:, :R])
        ctx.in_dtype = x.dtype
        return obj.to(x.dtype)

    @staticmethod
    def backward(ctx, g_obj):
        (grad_nr,) = ctx.saved_tensors
        gx = g_obj.to(torch.float32)[:, None] * grad_nr.T
        return gx.to(ctx.in_dtype), None


def fe_objective(problem: "pcls.Problem", x: torch.Tensor) -> torch.Tensor:
    """F(x) for restart rows x (R, n); differentiable in x."""
    return FEObjective.apply(x, problem)
