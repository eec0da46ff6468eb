"""Differentiable y = G(gamma) u: a torch.autograd.Function over ghost_apply / ghost_vjp.

Backward: the cotangent w of y pulls back to
    dL/du     = G^T w = G w        (G is symmetric: the transposed apply is the apply)
    dL/dgamma_j = w^T G_j u        (G is linear in gamma, §2.4 summed-penalty equation)
both computed by one fused HIP kernel (ghost_vjp).
"""

import torch


class GhostApply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, gamma, op):
        if gamma.device.type != "cuda" or gamma.dtype != torch.float64:
            raise ValueError("gamma must be a float64 CUDA tensor")
        g = gamma.detach().contiguous()
        op.set_gamma(g)
        y = op.apply(u.detach().contiguous())
        ctx.save_for_backward(u.detach(), g)
        ctx.op = op
        return y

    @staticmethod
    def backward(ctx, grad_y):
        u, g = ctx.saved_tensors
        op = ctx.op
        op.set_gamma(g)  # the context may have been re-used with another gamma since forward
        du, dg = op.vjp(u.contiguous(), grad_y.contiguous())
        return (du if ctx.needs_input_grad[0] else None,
                dg if ctx.needs_input_grad[1] else None, None)


def ghost_apply(u, gamma, op):
    """y = G(gamma) u, differentiable in u and gamma."""
    return GhostApply.apply(u, gamma, op)
