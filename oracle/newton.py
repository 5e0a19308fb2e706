"""Sequential Newton time march of the implicit scheme (oracle; test infrastructure only).

Defines the discrete solution of the backward Euler / BDF2 scheme of
Section 3.1 independently of any primal-dual iteration: for l = 0..N_t-1
solve  G(v) = (c0 v + c1 u^l + c2 u^{l-1}) / h_t + F(v) = 0  for v = u^{l+1}
by Newton's method started from u^l, with the exact Jacobian
c0/h_t I + dF/dv (a periodic tridiagonal matrix, solved directly).  This is
the per-step nonlinear solve that the primal-dual approach avoids (abstract,
Section 1), used here only as a reference.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fd
from .problem import Problem, time_coeffs


def march(prob: Problem, u0: np.ndarray, tol: float = 1e-14, max_newton: int = 50) -> np.ndarray:
    """Return u of shape (N_t+1, N_x) with u[0] = u0."""
    if prob.space == "dg_p2_llf":
        from . import dg
        return dg.p2_newton_march(prob, u0, tol, max_newton)
    if prob.space == "dg_p1_upwind":
        from . import dg1
        return dg1.p1_newton_march(prob, u0, tol, max_newton)
    nt, n, ht = prob.nt, prob.nx, prob.ht
    u = np.empty((nt + 1, n))
    u[0] = u0
    eye = sp.identity(n, format="csc")
    for l in range(nt):
        c0, c1, c2 = time_coeffs(prob.time, l)
        known = c1 * u[l] + (c2 * u[l - 1] if c2 != 0.0 else 0.0)
        v = u[l].copy()
        for _ in range(max_newton):
            g = (c0 * v + known) / ht + fd.flux_operator(prob, v)
            jac = ((c0 / ht) * eye + fd.flux_jacobian(prob, v)).tocsc()
            dv = spla.spsolve(jac, g)
            v -= dv
            if np.max(np.abs(dv)) <= tol * max(1.0, np.max(np.abs(v))):
                break
        u[l + 1] = v
    return u
