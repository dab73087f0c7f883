"""torch.autograd.Function around the S-build and its hand-written adjoint.

S = PronyS.apply(f, d, n, U, sigma, V) computes S_l = U^* T_l(f) V Sigma^{-1}
(l = 1..d) with prony_build_S; backward maps dL/dS to dL/df on the sample grid
with prony_build_S_adjoint. U, Sigma, V are constants of the map (they must not
require grad): the gradient describes the sensitivity of S_l to the samples.

BatchedPencil does the same for many instances at once: one batched S-build
(prony_build_S_batched) forward and one batched adjoint
(prony_build_S_adjoint_batched) backward, on the concatenated sample grids.
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
        ctx.f_shape = f.shape
        return S

    @staticmethod
    def backward(ctx, gS):
        U, sigma, V = ctx.saved_tensors
        gf = api.build_S_adjoint(gS.contiguous(), ctx.d, ctx.n, U, sigma, V, prec=ctx.prec_backward)
        return gf.view(ctx.f_shape), None, None, None, None, None, None, None


def pencil(f, d: int, n: int, U, sigma, V, prec_forward: str = "fp32", prec_backward: str = "fp32"):
    """Differentiable S_1..S_d of the sample grid f (shape (d, m, m))."""
    return PronyS.apply(f, d, n, U, sigma, V, prec_forward, prec_backward)


class _PronySBatched(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f_all, owner):
        owner._f_all.copy_(f_all.detach())
        owner.batch.run()
        ctx.owner = owner
        return owner._S_all.clone()

    @staticmethod
    def backward(ctx, gS_all):
        return ctx.owner.batch.adjoint(gS_all.contiguous()), None


class BatchedPencil:
    """Differentiable S-build of many instances with fixed factors.

    instances: sequence of (d, n, U, sigma, V) (U, V contiguous N x m complex128,
    no grad). Calling it on f_all, the sample grids of all instances concatenated
    in order (sum of gf_sizes complex128 values), returns S_all, the (d, m, m)
    matrices of all instances flattened and concatenated (sum of gs_sizes values);
    `split(S_all)` gives them back per instance. The forward runs in `prec`, and
    so does the adjoint (the batch's precision)."""

    def __init__(self, instances, prec: str = "fp32"):
        if not instances:
            raise ValueError("empty batch")
        dev = instances[0][2].device
        for d, n, U, sigma, V in instances:
            if U.requires_grad or V.requires_grad or sigma.requires_grad:
                raise ValueError("BatchedPencil differentiates with respect to f only; detach U, sigma and V")
        self.gf_sizes = [api.grid_size(d, n) for d, n, U, s, V in instances]
        self.gs_sizes = [d * U.shape[1] ** 2 for d, n, U, s, V in instances]
        self._f_all = torch.zeros(sum(self.gf_sizes), dtype=torch.complex128, device=dev)
        self._S_all = torch.empty(sum(self.gs_sizes), dtype=torch.complex128, device=dev)
        fs = torch.split(self._f_all, self.gf_sizes)
        Ss = [x.view(d, U.shape[1], U.shape[1]) for x, (d, n, U, s, V) in zip(torch.split(self._S_all, self.gs_sizes),
                                                                              instances)]
        self.batch = api.Batch([(d, n, f, U, s, V) for f, (d, n, U, s, V) in zip(fs, instances)], prec=prec,
                               outputs=Ss)
        self.shapes = self.batch.shapes

    def __call__(self, f_all):
        if f_all.numel() != self._f_all.numel():
            raise ValueError("f_all must hold sum(gf_sizes) values")
        return _PronySBatched.apply(f_all.reshape(-1), self)

    def split(self, S_all):
        return [x.view(d, m, m) for x, (d, n, m) in zip(torch.split(S_all, self.gs_sizes), self.shapes)]

    def close(self):
        self.batch.close()
