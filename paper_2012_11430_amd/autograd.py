"""torch.autograd.Function around the S-build and its hand-written adjoint.

S = PronyS.apply(f, d, n, U, sigma, V) computes S_l = U^* T_l(f) V Sigma^{-1}
(l = 1..d) with prony_build_S; backward maps dL/dS to dL/df on the sample grid
with prony_build_S_adjoint. U, Sigma, V are constants of the map (they must not
require grad): the gradient describes the sensitivity of S_l to the samples.
"""
from __future__ import annotations

import torch

from . import api


class PronyS(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, d: int, n: int, U, sigma, V, prec_forward: str = "fp32", prec_backward: str = "fp32"):
        if U.requires_grad or V.requires_grad or sigma.requires_grad:
            raise ValueError("PronyS differentiates with respect to f only; detach U, sigma and V")
        S = api.build_S(f.detach().contiguous(), d, n, U, sigma, V, prec=prec_forward)
        ctx.save_for_backward(U, sigma, V)
        ctx.d, ctx.n, ctx.prec_backward = d, n, prec_backward
        return S

    @staticmethod
    def backward(ctx, gS):
        U, sigma, V = ctx.saved_tensors
        gf = api.build_S_adjoint(gS.contiguous(), ctx.d, ctx.n, U, sigma, V, prec=ctx.prec_backward)
        return gf, None, None, None, None, None, None, None


def pencil(f, d: int, n: int, U, sigma, V, prec_forward: str = "fp32", prec_backward: str = "fp32"):
    """Differentiable S_1..S_d of the sample grid f (shape (d, m, m))."""
    return PronyS.apply(f, d, n, U, sigma, V, prec_forward, prec_backward)
