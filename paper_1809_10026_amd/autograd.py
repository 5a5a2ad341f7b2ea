"""torch.autograd wrappers: heat solve and space-time misfit.

HeatSolve maps (f, kappa) to u = A_kappa^{-1} B_kappa f with the library's
FD-preconditioned PCG; its backward pass solves the adjoint system with the
same solver (A_kappa is symmetric) and applies B_kappa^T and the kappa
derivative.  Only the forward solution u is kept for the backward pass (no
PCG iterates are stored).  Misfit maps u to (u - u*)^T M_Q (u - u*); the
library returns its gradient 2 M_Q (u - u*) with the loss.  Tensors are float64 CUDA vectors in colexicographic order; kappa is a
0-dim float64 tensor.  Every operator runs in the HIP library; torch only
scales the incoming gradient.
"""
from __future__ import annotations

import torch


class HeatSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, kappa, solver, rtol=1e-10, maxit=1000):
        solver.set_kappa(float(kappa))
        F = solver.load_apply(f.contiguous())
        u, it, rel = solver.solve(F, rtol=rtol, maxit=maxit)
        ctx.solver, ctx.rtol, ctx.maxit = solver, rtol, maxit
        ctx.save_for_backward(f, u, kappa)
        return u

    @staticmethod
    def backward(ctx, gu):
        f, u, kappa = ctx.saved_tensors
        S = ctx.solver
        S.set_kappa(float(kappa))
        lam, _, _ = S.solve(gu.contiguous(), rtol=ctx.rtol, maxit=ctx.maxit)
        gf = S.load_apply_T(lam) if ctx.needs_input_grad[0] else None
        gk = None
        if ctx.needs_input_grad[1]:
            gk = torch.tensor(S.dkappa(f.contiguous(), u, lam), dtype=kappa.dtype, device=kappa.device)
        return gf, gk, None, None, None


class Misfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, ustar, solver):
        loss, q = solver.misfit(u.contiguous(), ustar.contiguous())
        ctx.save_for_backward(q)
        return torch.tensor(loss, dtype=u.dtype, device=u.device)

    @staticmethod
    def backward(ctx, g):
        (q,) = ctx.saved_tensors
        return g * q, None, None


def heat_solve(f, kappa, solver, rtol=1e-10, maxit=1000):
    return HeatSolve.apply(f, kappa, solver, rtol, maxit)


def misfit(u, ustar, solver):
    return Misfit.apply(u, ustar, solver)
