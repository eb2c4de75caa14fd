"""torch.autograd.Function around the solve and its hand-written adjoint.

    x = EqSolveFn.apply(aP, aE, aW, aN, aS, aT, aB, b, x0, tol, maxit)

The tensors are float64 CUDA tensors shaped (nz, ny, nx).  Forward solves
A x = b (FP64 BiCGSTAB); backward, given w = dL/dx, solves A^T lambda = w with
the library's adjoint and returns dL/db = lambda and dL/da_k (P: -lambda*x;
neighbour slots: +lambda * x shifted to that neighbour, 0 out of the grid),
and None for x0, tol and maxit.
"""
from __future__ import annotations

import torch

from .solver import Context

_contexts = {}


def _context(shape, device):
    nz, ny, nx = shape
    key = (nx, ny, nz, device.index, torch.cuda.current_stream(device).cuda_stream)
    c = _contexts.get(key)
    if c is None:
        c = Context([(nx, ny, nz)], precision="fp64", device=device)
        _contexts[key] = c
    return c


class EqSolveFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, aP, aE, aW, aN, aS, aT, aB, b, x0, tol=1e-12, maxit=10000):
        diags = [t.contiguous() for t in (aP, aE, aW, aN, aS, aT, aB)]
        if b.dim() != 3:
            raise ValueError("EqSolveFn takes tensors shaped (nz, ny, nx)")
        c = _context(tuple(b.shape), b.device)
        x = (x0.detach().clone() if x0 is not None else torch.zeros_like(b)).contiguous()
        c.solve(diags, b.contiguous(), x, tol=tol, maxit=maxit)
        ctx.save_for_backward(*diags, x)
        ctx.tol, ctx.maxit = tol, maxit
        return x

    @staticmethod
    def backward(ctx, gx):
        *diags, x = ctx.saved_tensors
        c = _context(tuple(x.shape), x.device)
        gb, gd, _ = c.adjoint(diags, x, gx.contiguous(), tol=ctx.tol, maxit=ctx.maxit)
        return (*gd, gb, None, None, None)
