"""Preconditioner K_d of the dual proximal step (oracle; test infrastructure only).

The dual step of the G-prox PDHG (Section 2.2) is taken in the norm
||phi||_H^2 = ||d_t phi||^2 + c^2 ||d_x phi||^2 + ghat^2 ||d_xx phi||^2,
i.e. phi <- phi + tau_phi K^{-1} A(u) with
K = -d_tt - c^2 d_xx + ghat^2 d_xxxx (Section 2.2, linear case; the nonlinear case in the same section
drops the fourth-order term).  Section 3.3 takes K_d as a discretisation of
K and inverts it with the FFT.

Reading used here (the paper gives no stencil): K_d is the Gram form of the
discrete operators on the dual (row) space,

    K_d = (B_t B_t^T) (x) I_x  +  I_t (x) (c^2 L_x + ghat^2 L_x^2),

with B_t the time difference of the scheme acting on the unknown levels
(``fd.time_matrix``) and L_x the periodic (-1, 2, -1)/h_x^2 Laplacian.  For
backward Euler, B_t B_t^T = tridiag(-1; 1, 2, ..., 2; -1)/h_t^2: the discrete
||d_t phi||^2 with the terminal condition phi(T) = 0 (Section 3.1).  This
reading reproduces the iteration counts of Table 1.

Inversion: FFT along x diagonalises L_x (eigenvalues mu_k =
4 sin^2(pi k / N_x) / h_x^2); each Fourier mode then solves the banded system
(B_t B_t^T + s_k I) shat_k = rhat_k, s_k = c^2 mu_k + ghat^2 mu_k^2.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .fd import time_matrix
from .problem import Problem


def mode_shifts(prob: Problem) -> np.ndarray:
    """s_k for k = 0..N_x-1 (full FFT ordering)."""
    k = np.arange(prob.nx)
    mu = 4.0 * np.sin(np.pi * k / prob.nx) ** 2 / prob.hx ** 2
    return prob.precond_c ** 2 * mu + prob.precond_gamma_hat ** 2 * mu ** 2


def time_gram(prob: Problem) -> np.ndarray:
    """K_t = B_t B_t^T (dense N_t x N_t)."""
    b = time_matrix(prob)
    return b @ b.T


def kd_dense(prob: Problem) -> np.ndarray:
    """K_d assembled densely as Kronecker products (tiny grids only)."""
    n = prob.nx
    lx = (2.0 * np.eye(n) - np.roll(np.eye(n), 1, axis=1) - np.roll(np.eye(n), -1, axis=1)) / prob.hx ** 2
    sx = prob.precond_c ** 2 * lx + prob.precond_gamma_hat ** 2 * (lx @ lx)
    return np.kron(time_gram(prob), np.eye(n)) + np.kron(np.eye(prob.nt), sx)


def kd_solve(prob: Problem, r: np.ndarray) -> np.ndarray:
    """s = K_d^{-1} r for r of shape (N_t, N_x), via FFT in x and banded solves in t."""
    kt = time_gram(prob)
    nt = prob.nt
    # bandwidth of B_t B_t^T (no more off-diagonals than the matrix has)
    bw = min(2 if prob.time == "bdf2" else 1, nt - 1)
    # upper banded storage for solveh_banded: ab[bw + i - j, j] = a[i, j]
    ab0 = np.zeros((bw + 1, nt))
    for d in range(bw + 1):
        ab0[bw - d, d:] = np.diagonal(kt, d)
    rhat = np.fft.fft(r, axis=1)
    shat = np.empty_like(rhat)
    shifts = mode_shifts(prob)
    for k in range(prob.nx):
        ab = ab0.copy()
        ab[bw] += shifts[k]
        shat[:, k] = sla.solveh_banded(ab, rhat[:, k])
    return np.fft.ifft(shat, axis=1).real


# ------------------------------------------------------------------ full symbol
# Reading (beyond the paper, which drops the cross term d_t d_x of A^T A when it
# forms K in Section 2.2): K_full = J_c J_c^T with J_c = B_t (x) I + I (x) G_c the
# scheme's own Jacobian for the linear flux f(u) = c u (c the constant speed
# estimate; same Lax-Friedrichs constant, ghat in place of the viscosity).  G_c is
# circulant with symbol g_k, so per FFT mode K_k = L_k L_k^* with the lower
# triangular banded L_k = B_t + g_k I: one forward and one backward substitution.
def full_symbol(prob: Problem) -> np.ndarray:
    """g_k, k = 0..N_x-1: eigenvalues of the linear-flux spatial operator G_c."""
    th = 2.0 * np.pi * np.arange(prob.nx) / prob.nx
    c = prob.precond_c
    if prob.space == "fd_upwind":
        g = c * (1.0 - np.exp(-1j * th)) / prob.hx
    elif prob.space == "fd_lf":
        g = (1j * c * np.sin(th) + prob.lf_speed * (1.0 - np.cos(th))) / prob.hx
    else:
        raise ValueError("the full-symbol preconditioner covers the finite-difference fluxes")
    mu = 4.0 * np.sin(th / 2.0) ** 2 / prob.hx ** 2
    return g + prob.precond_gamma_hat * mu


def kd_full_solve(prob: Problem, r: np.ndarray) -> np.ndarray:
    """s = K_full^{-1} r for r of shape (N_t, N_x)."""
    b = time_matrix(prob)
    g = full_symbol(prob)
    rhat = np.fft.fft(r, axis=1)
    shat = np.empty_like(rhat)
    for k in range(prob.nx):
        L = b + g[k] * np.eye(prob.nt)
        y = sla.solve_triangular(L, rhat[:, k], lower=True)
        shat[:, k] = sla.solve_triangular(L.conj().T, y, lower=False)
    return np.fft.ifft(shat, axis=1).real


def kd_apply(prob: Problem, s: np.ndarray) -> np.ndarray:
    """K_d s (matrix-free; used to check kd_solve)."""
    kt = time_gram(prob)
    out = kt @ s
    c2, g2 = prob.precond_c ** 2, prob.precond_gamma_hat ** 2
    lap = (2.0 * s - np.roll(s, 1, axis=1) - np.roll(s, -1, axis=1)) / prob.hx ** 2
    lap2 = (2.0 * lap - np.roll(lap, 1, axis=1) - np.roll(lap, -1, axis=1)) / prob.hx ** 2
    return out + c2 * lap + g2 * lap2
