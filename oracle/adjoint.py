"""Gradient through the implicit scheme (oracle; test infrastructure only).

The converged saddle point satisfies A(U; u0) = 0 (Section 3.1: the primal
equation; at the saddle point the dual variable vanishes for a nonsingular
Jacobian).  For a loss l(u^0, U) the implicit-function theorem gives

    J(U)^T mu = dl/dU,     dl/du0 = dl/du^0 - (dA/du0)^T mu,

with dA/du0 nonzero only in row 0 (-1/h_t I, backward Euler start) and, for
BDF2, row 1 (+1/(2 h_t) I).  The solve J^T mu = g is the discrete dual
(backward-in-time) equation of Section 3.1 with a source term; here it is a
plain sparse direct solve, not a march.

For the DG schemes (Section 3.2: the P2 Legendre scheme with the local
Lax-Friedrichs flux, and the paper's P1 nodal upwind scheme) the unknowns of a
level are the cell coefficients (or nodal values), arrays (p, N_x), and J is
their exact Jacobian; the time coefficients act per coefficient, so the same
formula gives dl/du0 with respect to the initial coefficients.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import dg, dg1, fd
from .problem import Problem, time_coeffs


def _jacobian(prob: Problem, u: np.ndarray):
    if prob.space == "dg_p2_llf":
        return dg.p2_jacobian(prob, u)
    if prob.space == "dg_p1_upwind":
        return dg1.p1_jacobian(prob, u)
    return fd.jacobian(prob, u)


def adjoint_solve(prob: Problem, u: np.ndarray, g: np.ndarray) -> np.ndarray:
    """mu with J(u)^T mu = g[1:] (rows l = 0..N_t-1); g has the shape of u, (N_t+1, N_x) or
    (N_t+1, p, N_x) for DG."""
    J = _jacobian(prob, u).T.tocsc()
    shape = (prob.nt,) + tuple(np.shape(u)[1:])
    return spla.spsolve(J, np.asarray(g[1:], dtype=np.float64).ravel()).reshape(shape)


def gradient_u0(prob: Problem, u: np.ndarray, g: np.ndarray) -> np.ndarray:
    """dl/du0 given g = dl/du for every level (the shape of u)."""
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
