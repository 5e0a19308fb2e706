"""Gradient through the implicit scheme (oracle; test infrastructure only).

The converged saddle point satisfies A(U; u0) = 0 (Section 3.1: the primal
equation; at the saddle point the dual variable vanishes for a nonsingular
Jacobian).  For a loss l(u^0, U) the implicit-function theorem gives

    J(U)^T mu = dl/dU,     dl/du0 = dl/du^0 - (dA/du0)^T mu,

with dA/du0 nonzero only in row 0 (-1/h_t I, backward Euler start) and, for
BDF2, row 1 (+1/(2 h_t) I).  The solve J^T mu = g is the discrete dual
(backward-in-time) equation of Section 3.1 with a source term; here it is a
plain sparse direct solve, not a march.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import fd
from .problem import Problem, time_coeffs


def adjoint_solve(prob: Problem, u: np.ndarray, g: np.ndarray) -> np.ndarray:
    """mu with J(u)^T mu = g[1:] (rows l = 0..N_t-1); g has shape (N_t+1, N_x)."""
    J = fd.jacobian(prob, u).T.tocsc()
    return spla.spsolve(J, np.asarray(g[1:], dtype=np.float64).ravel()).reshape(prob.nt, prob.nx)


def gradient_u0(prob: Problem, u: np.ndarray, g: np.ndarray) -> np.ndarray:
    """dl/du0 given g = dl/du for every level (shape (N_t+1, N_x))."""
    mu = adjoint_solve(prob, u, g)
    grad = np.array(g[0], dtype=np.float64)
    for row in (0, 1):
        if row >= prob.nt:
            break
        c0, c1, c2 = time_coeffs(prob.time, row)
        coef = c1 if row == 0 else c2       # coefficient of u^0 in this row
        grad -= (coef / prob.ht) * mu[row]
    return grad


def terminal_loss(prob: Problem, u: np.ndarray, target: np.ndarray) -> float:
    """l = h_x sum_j (u^{N_t}_j - target_j)^2 (discrete L2, Section 2.2 weights)."""
    d = u[-1] - target
    return float(prob.hx * np.sum(d * d))


def terminal_loss_grad(prob: Problem, u: np.ndarray, target: np.ndarray) -> np.ndarray:
    """dl/du for the terminal loss: nonzero only at level N_t."""
    g = np.zeros_like(u)
    g[-1] = 2.0 * prob.hx * (u[-1] - target)
    return g
