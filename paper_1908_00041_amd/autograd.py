"""Differentiable forward and adjoint VSHT for torch.autograd.

Both transforms are linear maps, so each backward is the Hermitian transpose
of its forward, and both transposes are themselves transforms of the library:

* AdjointVSHT: T = S(a, b), the adjoint of eq. (SLvec), with S the synthesis
  matrix [Y^div | Y^curl] at the plan's points.  Backward:
  (grad_a, grad_b) = S^H grad_T, the forward transform of eq. (fwdvsht2) with
  unit weights.
* ForwardVSHT: (a, b) = S^H W T, eq. (fwdvsht2) with the quadrature weights
  W = diag(w).  Backward: grad_T = W S (grad_a, grad_b), the adjoint
  transform with every output point multiplied by its weight.

Gradients follow PyTorch's convention for complex tensors (for a real loss,
the gradient of z is dL/dRe z + i dL/dIm z, and a linear map y = A x sends the
output gradient g to A^H g).  Leading batch dimensions are allowed: a, b of
shape (..., K) and T of shape (..., n, 3); every field runs through the same
plan.  No arithmetic of the transforms happens here: each direction is one
call of the C library.
"""
import torch


class AdjointVSHT(torch.autograd.Function):
    """T = Adj(a, b) at the plan's points; backward = unit-weight forward transform."""

    @staticmethod
    def forward(ctx, plan, a, b):
        ctx.plan = plan
        return plan.adjoint_many(a, b)

    @staticmethod
    def backward(ctx, gT):
        ga, gb = ctx.plan.forward_many(gT.contiguous(), unit_weights=True)
        return None, ga, gb


class ForwardVSHT(torch.autograd.Function):
    """(a, b) = Fwd(T) with the plan's quadrature weights; backward = weighted adjoint."""

    @staticmethod
    def forward(ctx, plan, T):
        ctx.plan = plan
        return plan.forward_many(T)

    @staticmethod
    def backward(ctx, ga, gb):
        plan = ctx.plan
        if ga is None:
            ga = torch.zeros_like(gb)
        if gb is None:
            gb = torch.zeros_like(ga)
        return None, plan.adjoint_many(ga.contiguous(), gb.contiguous(), times_weights=True)


def adjoint_vsht(plan, a, b):
    """Differentiable adjoint transform (a, b (..., K) -> T (..., n, 3))."""
    return AdjointVSHT.apply(plan, a, b)


def forward_vsht(plan, T):
    """Differentiable forward transform (T (..., n, 3) -> a, b (..., K))."""
    return ForwardVSHT.apply(plan, T)
