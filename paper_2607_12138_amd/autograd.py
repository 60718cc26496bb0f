"""Differentiable mass solve x = M(rho)^-1 b for H1 elements with a
piecewise-constant density (M_K = rho_K |det J_K| Mhat, eq. h1_mass_pullback).

backward: with g = dL/dx, the adjoint lambda = M^-1 g (M symmetric, the
same BRAS-preconditioned CG), dL/db = lambda and
dL/drho_K = -lambda_K^T (dM_K/drho_K) x_K computed by the library's
per-element contraction.

The problem object holds one density at a time.  forward() saves the density
it solved with; backward() re-installs it when another solve has changed the
problem's density in between (several losses, checkpointing, probes), so the
adjoint always uses the operator of its own forward solve.
"""
import torch

from . import _lib as L


class BrasMassSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, b, rho, problem, rtol=1e-10, maxit=5000):
        rho_c = rho.detach().contiguous().clone()
        problem.set_density(rho_c)
        x, st, its, rel = problem.solve(b.detach().contiguous(), pc="bras", rtol=rtol, maxit=maxit)
        if st != L.BRAS_OK:
            raise L.BrasError(st, "forward solve: " + L.bras_last_error())
        ctx.problem = problem
        ctx.rtol, ctx.maxit = rtol, maxit
        ctx.save_for_backward(x, rho_c)
        ctx.forward_iters = its
        return x

    @staticmethod
    def backward(ctx, gx):
        x, rho = ctx.saved_tensors
        problem = ctx.problem
        cur = problem.rho_d
        if cur is None or (cur.data_ptr() != rho.data_ptr() and not torch.equal(cur, rho)):
            problem.set_density(rho)
        lam, st, its, rel = problem.solve(gx.detach().contiguous(), pc="bras", rtol=ctx.rtol, maxit=ctx.maxit)
        if st != L.BRAS_OK:
            raise L.BrasError(st, "adjoint solve: " + L.bras_last_error())
        grho = problem.rho_grad(x, lam)
        return lam, grho, None, None, None


def mass_solve(b, rho, problem, rtol=1e-10, maxit=5000):
    return BrasMassSolve.apply(b, rho, problem, rtol, maxit)
