"""J(u_hat, T) as a torch.autograd.Function whose backward is the hand-written adjoint kernel.

    J = LoopCost.apply(uhat, T, L)              # uhat: (nloops, Ns, Nx//2+1) or (Ns, Nx//2+1)
                                                # complex128 (rfft layout); T: (nloops,) float64
    J = LoopCostBand.apply(ub, T, L, Nx, Ns)    # ub: (nloops, C, NB) complex128 (band layout)

The forward is loop_cost_fwd: J, dJ/dT and the band residual r_hat, which the context keeps.
The backward is loop_cost_bwd: it applies the adjoint operator to the saved residual and
returns the gradient in torch's complex convention, d/dRe + i d/dIm, which is -w_j L G_1 in
the band, and dJ/dT for the periods (Sec. 3, eq. KS_G with J halved). By default the backward
recomputes u on the s grid from u_hat, so the context holds only state-sized tensors and no
transform intermediate. save_u=True keeps that intermediate from the forward instead
(nloops x C x Ns complex values, 1.5 times the band state at 256 x 1024) and saves the
backward one column transform. Both give the same gradient bit for bit.
"""
from __future__ import annotations

import torch

from . import api


def _usave(ctx, nl, Nx, Ns, device, save_u):
    if save_u and any(ctx.needs_input_grad[:2]):
        return api.saved_u(nl, Nx, Ns, device)
    return None


class LoopCost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, uhat, T, L, save_u=False):
        uhat = uhat.contiguous()
        T = T.contiguous()
        ctx.L = float(L)
        nl, Nx, Ns = api.shape_of(uhat)
        us = _usave(ctx, nl, Nx, Ns, uhat.device, save_u)
        J, dJdT, rsave = api.loop_cost_fwd(uhat, T, L, usave=us)
        ctx.has_u = us is not None
        ctx.save_for_backward(uhat, T, rsave, dJdT, *((us,) if us is not None else ()))
        return J

    @staticmethod
    def backward(ctx, gJ):
        uhat, T, rsave, dJdT, *us = ctx.saved_tensors
        gu, gT = api.loop_cost_bwd(uhat, T, ctx.L, rsave, dJdT, gJ.contiguous().to(torch.float64),
                                   usave=us[0] if ctx.has_u else None)
        return gu, gT, None, None


class LoopCostBand(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ub, T, L, Nx, Ns, save_u=False):
        ub = ub.contiguous()
        T = T.contiguous()
        ctx.L, ctx.grid = float(L), (int(Nx), int(Ns))
        us = _usave(ctx, api.band_shape_of(ub, int(Nx), int(Ns)), int(Nx), int(Ns), ub.device, save_u)
        J, dJdT, rsave = api.loop_cost_fwd(ub, T, L, layout=api.LAYOUT_BAND, grid=ctx.grid, usave=us)
        ctx.has_u = us is not None
        ctx.save_for_backward(ub, T, rsave, dJdT, *((us,) if us is not None else ()))
        return J

    @staticmethod
    def backward(ctx, gJ):
        ub, T, rsave, dJdT, *us = ctx.saved_tensors
        gu, gT = api.loop_cost_bwd(ub, T, ctx.L, rsave, dJdT, gJ.contiguous().to(torch.float64),
                                   layout=api.LAYOUT_BAND, grid=ctx.grid, usave=us[0] if ctx.has_u else None)
        return gu, gT, None, None, None, None


def loop_cost(uhat, T, L, save_u=False):
    """Differentiable J = 1/2 int int r^2 per loop (rfft layout)."""
    return LoopCost.apply(uhat, T, L, save_u)


def loop_cost_band(ub, T, L, Nx, Ns, save_u=False):
    """Differentiable J = 1/2 int int r^2 per loop (band layout)."""
    return LoopCostBand.apply(ub, T, L, Nx, Ns, save_u)
