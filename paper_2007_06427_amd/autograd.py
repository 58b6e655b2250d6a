"""J(u_hat, T) as a torch.autograd.Function whose backward is the hand-written adjoint kernel.

    J = LoopCost.apply(uhat, T, L)      # uhat: (nloops, Ns, Nx//2+1) or (Ns, Nx//2+1) complex128
                                        # T: (nloops,) float64; J: (nloops,) float64

The forward is loop_cost. The backward calls loop_cost_grad, which recomputes the transforms
from (u_hat, T) (nothing of the forward's intermediates is stored). It returns the
gradient in torch's complex convention, d/dRe + i d/dIm, which is -w_j L G_1 in the band, and
dJ/dT for the periods (Sec. 3, eq. KS_G with J halved).
"""
from __future__ import annotations

import torch

from . import api


class LoopCost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, uhat, T, L):
        uhat = uhat.contiguous()
        T = T.contiguous()
        ctx.L = float(L)
        ctx.squeeze = uhat.dim() == 2
        ctx.save_for_backward(uhat, T)
        return api.loop_cost(uhat, T, L)

    @staticmethod
    def backward(ctx, gJ):
        uhat, T = ctx.saved_tensors
        gu, gT = api.loop_cost_grad(uhat, T, ctx.L, gJ.contiguous().to(torch.float64))
        return gu, gT, None


def loop_cost(uhat, T, L):
    """Differentiable J = 1/2 int int r^2 per loop."""
    return LoopCost.apply(uhat, T, L)
