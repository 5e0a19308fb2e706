"""Differentiable space-time solve: d loss / d u0 by the implicit-function adjoint.

Forward: Algorithm 1 (pdhg_solve) to the requested residual; returns u at
every level, shape (nt+1, nx).  Backward: the converged u solves the implicit
scheme A(u; u0) = 0 (Section 3.1), so for a loss l(u) the gradient with
respect to u0 is dl/du^0 - (dA/du0)^T mu with J(u)^T mu = dl/du.  J^T is the
dual-equation operator obtained by summation by parts (Section 3.1); the
library solves it by a backward march in time (pdhg_adjoint, mode SOLVE), one
periodic tridiagonal system per level.  No primal-dual iterate is stored:
only the converged u is kept for the backward pass.

The gradient is that of the implicit scheme's solution map; it equals the
derivative of the returned PDHG iterate up to the solve tolerance.
"""
from __future__ import annotations

import warnings

import torch


class PDHGSolve(torch.autograd.Function):
    """u = PDHGSolve.apply(u0, solver, solve_kwargs) with u of shape (nt+1, nx)."""

    @staticmethod
    def forward(ctx, u0, solver, solve_kwargs, allow_unconverged=False):
        res = solver.solve(u0.detach().contiguous(), **(solve_kwargs or {}))
        if res.status < 0 or res.status == 2:
            raise RuntimeError(f"PDHG solve failed (status {res.status}): {res.stats}")
        if res.status == 1:
            # the implicit-function adjoint is the derivative of the solution of A(u) = 0; an iterate
            # stopped by max_iter is not that solution
            msg = (f"PDHG solve stopped at max_iter={res.stats['iters']} with ||A(u)|| = "
                   f"{res.stats['res_primal']:.3e} above eps; the adjoint gradient assumes A(u) = 0")
            if not allow_unconverged:
                raise RuntimeError(msg + " (pass allow_unconverged=True to accept it)")
            warnings.warn(msg, RuntimeWarning, stacklevel=2)
        ctx.solver = solver
        ctx.stats = res.stats
        ctx.save_for_backward(res.u)
        return res.u

    @staticmethod
    def backward(ctx, g_u):
        (u,) = ctx.saved_tensors
        grad = ctx.solver.adjoint_solve(u, g_u.contiguous())
        return grad, None, None, None


def solve(u0, solver, allow_unconverged: bool = False, **solve_kwargs):
    """Differentiable solve; see PDHGSolve.  A solve that ends at max_iter raises unless
    allow_unconverged (then it warns); one that stalls at the rounding floor (PDHG_STALLED, the
    single-precision stop rule) is accepted."""
    return PDHGSolve.apply(u0, solver, solve_kwargs, allow_unconverged)
