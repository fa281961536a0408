"""torch.autograd.Function around the preconditioner solve Z = L^-T L^-1 R.

Forward runs icpcg_apply (two triangular solves); backward runs
icpcg_apply_backward (two transposed solves and the pattern pass for dL). This
is the differentiation a learned correction of L (Eq. (2),
L = L_IC + GNN(A)) needs to train through the preconditioner.
"""

from __future__ import annotations

import torch

from .solver import Preconditioner


class PrecApply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, l_val: torch.Tensor, R: torch.Tensor, prec: Preconditioner):
        prec.update_values(l_val.detach())
        Y, Z = prec.apply(R.detach())
        ctx.save_for_backward(Y, Z)
        ctx.prec = prec
        ctx.version = prec.version
        ctx.l_dtype = l_val.dtype
        ctx.r_dtype = R.dtype
        return Z

    @staticmethod
    def backward(ctx, G: torch.Tensor):
        Y, Z = ctx.saved_tensors
        if ctx.prec.version != ctx.version:
            raise RuntimeError("the preconditioner's values changed between forward and backward")
        dR, dL = ctx.prec.apply_backward(G, Y, Z)
        return dL.to(ctx.l_dtype), dR.to(ctx.r_dtype), None


def prec_apply(l_val: torch.Tensor, R: torch.Tensor, prec: Preconditioner) -> torch.Tensor:
    """Differentiable Z = L^-T L^-1 R with respect to L's stored values and R."""
    return PrecApply.apply(l_val, R, prec)
