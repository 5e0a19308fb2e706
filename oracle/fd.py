"""Finite-difference space-time residual and its Jacobian (oracle; test infrastructure only).

Notation (Sections 3.1-3.2): levels l = 0..N_t with u^0 = u0 held fixed;
the unknowns are U = (u^1, ..., u^{N_t}); grid points x_j = j h_x,
j = 0..N_x-1, periodic.  One implicit equation per row l = 0..N_t-1:

    A(u)^l = (c0 u^{l+1} + c1 u^l + c2 u^{l-1}) / h_t + F(u^{l+1})

(backward Euler / BDF2 coefficients from ``problem.time_coeffs``).  The
spatial operator F is one of

* first-order upwind difference of the flux, F_j = (f(v_j) - f(v_{j-1}))/h_x
  (assumes f' >= 0, as in Section 3.2.2 and Section 4.3);
* global Lax-Friedrichs: fhat_{j+1/2} = (f(v_j)+f(v_{j+1}))/2
  - lf (v_{j+1}-v_j)/2, F_j = (fhat_{j+1/2} - fhat_{j-1/2})/h_x;
* plus centred diffusion -gamma (v_{j+1} - 2 v_j + v_{j-1})/h_x^2 when gamma > 0;
* or, for the variable-coefficient heat equation (Section 3.2.1),
  F_j = -Lap(v)_j with gamma_{j+-1/2} = gamma((j +- 1/2) h_x).

The Jacobian J = dA/dU is assembled as an explicit sparse matrix from the
entry-wise derivatives of these formulas; J^T is its exact transpose.  This
is the summation-by-parts "dual equation" operator of Section 3.1
(the forward-Euler-like sweep for phi): J(u)^T phi evaluated row by row.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .problem import Problem, time_coeffs


# ---------------------------------------------------------------- spatial operator
def _heat_gammas(prob: Problem):
    x = np.arange(prob.nx, dtype=np.float64) * prob.hx
    gp = prob.gamma_fn(x + 0.5 * prob.hx)   # gamma_{j+1/2}
    gm = prob.gamma_fn(x - 0.5 * prob.hx)   # gamma_{j-1/2}
    return gp, gm


def flux_operator(prob: Problem, v: np.ndarray) -> np.ndarray:
    """F(v) for one time level (periodic), float64."""
    hx = prob.hx
    vp = np.roll(v, -1)   # v_{j+1}
    vm = np.roll(v, 1)    # v_{j-1}
    if prob.space == "fd_upwind":
        out = (prob.f(v) - prob.f(vm)) / hx
    elif prob.space == "fd_lf":
        fh_plus = 0.5 * (prob.f(v) + prob.f(vp)) - 0.5 * prob.lf_speed * (vp - v)
        fh_minus = np.roll(fh_plus, 1)
        out = (fh_plus - fh_minus) / hx
    elif prob.space == "heat_var":
        gp, gm = _heat_gammas(prob)
        return -(gp * (vp - v) - gm * (v - vm)) / (hx * hx)
    else:
        raise ValueError(f"fd oracle does not handle space={prob.space!r}")
    if prob.gamma != 0.0:
        out = out - prob.gamma * (vp - 2.0 * v + vm) / (hx * hx)
    return out


def flux_jacobian_diags(prob: Problem, v: np.ndarray):
    """Stencil of dF/dv: arrays (lo, di, up) with dF_j = lo_j dv_{j-1} + di_j dv_j + up_j dv_{j+1}.

    Works on one level (shape (N_x,)) or a stack of levels (shape (L, N_x)).
    """
    hx = prob.hx
    vp = np.roll(v, -1, axis=-1)
    vm = np.roll(v, 1, axis=-1)
    zero = np.zeros_like(v)
    if prob.space == "fd_upwind":
        lo, di, up = -prob.fp(vm) / hx, prob.fp(v) / hx, zero
    elif prob.space == "fd_lf":
        lf = prob.lf_speed
        lo = (-0.5 * prob.fp(vm) - 0.5 * lf) / hx
        di = zero + lf / hx
        up = (0.5 * prob.fp(vp) - 0.5 * lf) / hx
    elif prob.space == "heat_var":
        gp, gm = _heat_gammas(prob)
        h2 = hx * hx
        return zero - gm / h2, zero + (gp + gm) / h2, zero - gp / h2
    else:
        raise ValueError(prob.space)
    if prob.gamma != 0.0:
        g = prob.gamma / (hx * hx)
        lo, di, up = lo - g, di + 2.0 * g, up - g
    return lo, di, up


def _stencil_coo(lo, di, up, n, row0=0, col0=0):
    j = np.arange(n)
    rows = np.concatenate([j, j, j]) + row0
    cols = np.concatenate([(j - 1) % n, j, (j + 1) % n]) + col0
    return rows, cols, np.concatenate([lo, di, up])


def flux_jacobian(prob: Problem, v: np.ndarray) -> sp.csr_matrix:
    """dF/dv as a sparse periodic N_x x N_x matrix: entry (j, k) = dF_j/dv_k.

    Duplicate (row, column) pairs, which occur for N_x <= 2, are summed.
    """
    n = prob.nx
    r, c, x = _stencil_coo(*flux_jacobian_diags(prob, v), n)
    return sp.coo_matrix((x, (r, c)), shape=(n, n)).tocsr()


# ---------------------------------------------------------------- space-time operator
def residual(prob: Problem, u: np.ndarray) -> np.ndarray:
    """A(u): array (N_t, N_x); u is the full array (N_t+1, N_x) including u^0."""
    nt, ht = prob.nt, prob.ht
    r = np.empty((nt, prob.nx))
    for l in range(nt):
        c0, c1, c2 = time_coeffs(prob.time, l)
        t = c0 * u[l + 1] + c1 * u[l]
        if c2 != 0.0:
            t = t + c2 * u[l - 1]
        r[l] = t / ht + flux_operator(prob, u[l + 1])
    return r


def jacobian(prob: Problem, u: np.ndarray) -> sp.csr_matrix:
    """J = dA/dU, sparse (N_t N_x) x (N_t N_x).

    Row block l, column block m-1 (unknown u^m, m = 1..N_t).  u^0 is fixed
    and carries no column.  Row block l holds c0/h_t I + dF(u^{l+1}) in
    column block l, c1/h_t I in column block l-1 and c2/h_t I in column
    block l-2 (when those unknown levels exist).
    """
    nt, n, ht = prob.nt, prob.nx, prob.ht
    lo, di, up = flux_jacobian_diags(prob, u[1:])
    rows, cols, vals = [], [], []
    j = np.arange(n)
    for l in range(nt):
        c0, c1, c2 = time_coeffs(prob.time, l)
        r, c, x = _stencil_coo(lo[l], di[l] + c0 / ht, up[l], n, l * n, l * n)
        rows.append(r); cols.append(c); vals.append(x)
        if l >= 1 and c1 != 0.0:
            rows.append(l * n + j); cols.append((l - 1) * n + j); vals.append(np.full(n, c1 / ht))
        if l >= 2 and c2 != 0.0:
            rows.append(l * n + j); cols.append((l - 2) * n + j); vals.append(np.full(n, c2 / ht))
    size = nt * n
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(size, size)).tocsr()


def apply_jt(prob: Problem, u: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """J(u)^T phi, returned as (N_t, N_x) indexed by unknown level m-1."""
    return (jacobian(prob, u).T @ phi.ravel()).reshape(prob.nt, prob.nx)


def apply_j(prob: Problem, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """J(u) v for v indexed like the unknowns (N_t, N_x)."""
    return (jacobian(prob, u) @ v.ravel()).reshape(prob.nt, prob.nx)


def wnorm(prob: Problem, z: np.ndarray) -> float:
    """Space-time L2 norm sqrt(h_t h_x sum z^2) (the L2 norm of Section 2.2 on the grid)."""
    return float(np.sqrt(prob.ht * prob.hx * np.sum(np.asarray(z, dtype=np.float64) ** 2)))


def time_matrix(prob: Problem) -> np.ndarray:
    """Dense B_t (N_t x N_t): the time difference acting on the unknown levels.

    Row l, column m-1 holds the coefficient of u^m in row l of A, divided by
    h_t; the u^0 terms move to the right-hand side.
    """
    nt, ht = prob.nt, prob.ht
    b = np.zeros((nt, nt))
    for l in range(nt):
        c0, c1, c2 = time_coeffs(prob.time, l)
        b[l, l] = c0 / ht
        if l >= 1:
            b[l, l - 1] = c1 / ht
        if l >= 2:
            b[l, l - 2] = c2 / ht
    return b


def mass(prob: Problem, u: np.ndarray) -> np.ndarray:
    """Discrete mass h_x sum_j u^l_j per level."""
    return prob.hx * np.sum(u, axis=-1)
