"""J(u_hat, T) as a torch.autograd.Function whose backward is the hand-written adjoint kernel.

    J = LoopCost.apply(uhat, T, L)              # uhat: (nloops, Ns, Nx//2+1) or (Ns, Nx//2+1)
                                                # complex128 (rfft layout); T: (nloops,) float64
    J = LoopCostBand.apply(ub, T, L, Nx, Ns)    # ub: (nloops, C, NB) complex128 (band layout)

The forward is loop_cost_fwd: J, dJ/dT and the band residual r_hat, which the context keeps
(the size of the state; no transform intermediate is stored). The backward is loop_cost_bwd:
it recomputes u on the grid, applies the adjoint operator to the saved residual and returns
the gradient in torch's complex convention, d/dRe + i d/dIm, which is -w_j L G_1 in the band,
and dJ/dT for the periods (Sec. 3, eq. KS_G with J halved).
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
        J, dJdT, rsave = api.loop_cost_fwd(uhat, T, L)
        ctx.save_for_backward(uhat, T, rsave, dJdT)
        return J

    @staticmethod
    def backward(ctx, gJ):
        uhat, T, rsave, dJdT = ctx.saved_tensors
        gu, gT = api.loop_cost_bwd(uhat, T, ctx.L, rsave, dJdT, gJ.contiguous().to(torch.float64))
        return gu, gT, None


class LoopCostBand(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ub, T, L, Nx, Ns):
        ub = ub.contiguous()
        T = T.contiguous()
        ctx.L, ctx.grid = float(L), (int(Nx), int(Ns))
        J, dJdT, rsave = api.loop_cost_fwd(ub, T, L, layout=api.LAYOUT_BAND, grid=ctx.grid)
        ctx.save_for_backward(ub, T, rsave, dJdT)
        return J

    @staticmethod
    def backward(ctx, gJ):
        ub, T, rsave, dJdT = ctx.saved_tensors
        gu, gT = api.loop_cost_bwd(ub, T, ctx.L, rsave, dJdT, gJ.contiguous().to(torch.float64),
                                   layout=api.LAYOUT_BAND, grid=ctx.grid)
        return gu, gT, None, None, None


def loop_cost(uhat, T, L):
    """Differentiable J = 1/2 int int r^2 per loop (rfft layout)."""
    return LoopCost.apply(uhat, T, L)


def loop_cost_band(ub, T, L, Nx, Ns):
    """Differentiable J = 1/2 int int r^2 per loop (band layout)."""
    return LoopCostBand.apply(ub, T, L, Nx, Ns)
