"""DG P2 discretisation in space (oracle; test infrastructure only).

Discontinuous Galerkin with a Legendre basis of degree 2 on N_x uniform
periodic cells I_j = [j h, (j+1) h] (Section 3.2 builds DG from the weak form
on each cell; the paper's own example is P1 with an upwind flux, this is the
P2 / local Lax-Friedrichs variant of the same construction):

    xi = 2 (x - x_j) / h,  x_j the cell centre;  P_0 = 1, P_1 = xi, P_2 = (3 xi^2 - 1) / 2
    u_h = sum_k v_jk P_k(xi) on I_j;   mass  int_{I_j} P_k P_m dx = h / (2k+1) delta_km

Weak form per cell and test function P_k, divided by the mass:

    dv_jk/dt + F_jk(v) = 0,
    F_jk = -(2k+1)/h ( V_jk - fhat_{j+1/2} + (-1)^k fhat_{j-1/2} ),
    V_jk = int_{-1}^{1} f(u_h(xi)) P_k'(xi) dxi        (3-point Gauss: exact for quadratic f)

with the traces a_j = u_h(x_{j+1/2}^-) = v_j0 + v_j1 + v_j2 (right edge of cell j),
b_j = u_h(x_{j-1/2}^+) = v_j0 - v_j1 + v_j2 (left edge of cell j), and the local
Lax-Friedrichs flux at x_{j+1/2} between a = a_j and b = b_{j+1}:

    fhat(a, b) = (f(a) + f(b)) / 2 - s (b - a) / 2,   s = max(|f'(a)|, |f'(b)|)

(tie |f'(a)| = |f'(b)| takes a's branch for the generalised derivative).
The implicit scheme in time is that of Section 3.1 (fd.time_coeffs), applied
coefficient-wise: A_jk^l = (c0 v^{l+1} + c1 v^l + c2 v^{l-1})_jk / h_t + F_jk(v^{l+1}).

Arrays: u [N_t+1][3][N_x] (coefficient planes), residual and phi [N_t][3][N_x].
Norm of a space-time array: the coefficient norm sqrt(h_t h_x sum z^2), as for
finite differences.

Preconditioner (Section 2.2 / 3.3 with the Gram reading used for finite
differences): K_d = (B_t B_t^T) (x) I + I_t (x) c^2 G G^T, G the unit-speed upwind
DG operator (the linear-flux case of F above, a block-circulant matrix with
blocks G_0 on the diagonal and G_-1 below it).  In Fourier over the cells G has
the 3x3 symbol G(theta) = G_0 + G_-1 e^{-i theta}; c^2 G G^* = Q Lambda Q^* per mode,
and each eigen-branch solves (B_t B_t^T + lambda) z = (Q^* rhat) along t.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fd import time_matrix, wnorm
from .problem import Problem, time_coeffs

GAUSS3_X = np.array([-np.sqrt(3.0 / 5.0), 0.0, np.sqrt(3.0 / 5.0)])
GAUSS3_W = np.array([5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0])


def legendre(xi):
    """(P_0, P_1, P_2) at xi, stacked on the first axis."""
    xi = np.asarray(xi, dtype=np.float64)
    return np.stack([np.ones_like(xi), xi, 0.5 * (3.0 * xi * xi - 1.0)])


def dlegendre(xi):
    """(P_0', P_1', P_2') with respect to xi."""
    xi = np.asarray(xi, dtype=np.float64)
    return np.stack([np.zeros_like(xi), np.ones_like(xi), 3.0 * xi])


def p2_project(fn, nx: int, length: float = 1.0, npts: int = 8) -> np.ndarray:
    """L2 projection of fn onto P2 per cell: v_jk = (2k+1)/2 int_{-1}^{1} fn(x(xi)) P_k(xi) dxi,
    by npts-point Gauss-Legendre quadrature.  Returns (3, nx)."""
    h = length / nx
    xq, wq = np.polynomial.legendre.leggauss(npts)
    centres = (np.arange(nx) + 0.5) * h
    x = centres[None, :] + 0.5 * h * xq[:, None]          # (npts, nx)
    fx = fn(x)
    P = legendre(xq)                                      # (3, npts)
    out = np.einsum("kq,q,qj->kj", P, wq, fx)
    return out * ((2.0 * np.arange(3) + 1.0) / 2.0)[:, None]


def evaluate(v: np.ndarray, xi) -> np.ndarray:
    """u_h at local coordinate(s) xi in every cell: (..., nx)."""
    return np.einsum("k...,kj->...j", legendre(xi), v)


def traces(v: np.ndarray):
    """(a, b): right-edge values a_j and left-edge values b_j of every cell."""
    return v[0] + v[1] + v[2], v[0] - v[1] + v[2]


def llf_flux(prob: Problem, a, b):
    s = np.maximum(np.abs(prob.fp(a)), np.abs(prob.fp(b)))
    return 0.5 * (prob.f(a) + prob.f(b)) - 0.5 * s * (b - a)


def llf_partials(prob: Problem, a, b):
    """Generalised derivatives (d fhat / da, d fhat / db)."""
    fa, fb = prob.fp(a), prob.fp(b)
    s = np.maximum(np.abs(fa), np.abs(fb))
    f2 = 2.0 * prob.alpha
    a_branch = np.abs(fa) >= np.abs(fb)
    sa = np.where(a_branch, np.sign(fa) * f2, 0.0)
    sb = np.where(a_branch, 0.0, np.sign(fb) * f2)
    da = 0.5 * fa + 0.5 * s - 0.5 * (b - a) * sa
    db = 0.5 * fb - 0.5 * s - 0.5 * (b - a) * sb
    return da, db


def volume_term(prob: Problem, v: np.ndarray) -> np.ndarray:
    """V_jk = int f(u_h) P_k' dxi by 3-point Gauss.  (3, nx)."""
    uq = evaluate(v, GAUSS3_X)                            # (3 nodes, nx)
    return np.einsum("q,kq,qj->kj", GAUSS3_W, dlegendre(GAUSS3_X), prob.f(uq))


def spatial_operator(prob: Problem, v: np.ndarray) -> np.ndarray:
    """F(v) of shape (3, nx)."""
    h = prob.hx
    a, b = traces(v)
    fr = llf_flux(prob, a, np.roll(b, -1))                # fhat_{j+1/2}
    fl = np.roll(fr, 1)                                   # fhat_{j-1/2}
    V = volume_term(prob, v)
    k = np.arange(3)[:, None]
    return -((2.0 * k + 1.0) / h) * (V - fr[None, :] + ((-1.0) ** k) * fl[None, :])


def spatial_blocks(prob: Problem, v: np.ndarray):
    """3x3 blocks of dF/dv per cell: (D, L, U) with F_j depending on v_j (D_j), v_{j-1} (L_j)
    and v_{j+1} (U_j).  Each of shape (nx, 3, 3), [j, k, m] = dF_jk / dv_{., m}."""
    h, nx = prob.hx, prob.nx
    a, b = traces(v)
    ar, bl = a, np.roll(b, -1)                           # interface j+1/2: (a_j, b_{j+1})
    da_r, db_r = llf_partials(prob, ar, bl)
    da_l, db_l = np.roll(da_r, 1), np.roll(db_r, 1)       # interface j-1/2: (a_{j-1}, b_j)
    uq = evaluate(v, GAUSS3_X)                            # (q, nx)
    fpq = prob.fp(uq)
    Pq, dPq = legendre(GAUSS3_X), dlegendre(GAUSS3_X)     # (3, q)
    dV = np.einsum("q,kq,mq,qj->jkm", GAUSS3_W, dPq, Pq, fpq)   # dV_jk / dv_jm
    k = np.arange(3)
    sk = (-1.0) ** k                                      # (-1)^k, also d b / d v_m
    scale = -((2.0 * k + 1.0) / h)                        # per row k
    ones = np.ones(3)
    D = dV - da_r[:, None, None] * ones[None, None, :] + sk[None, :, None] * db_l[:, None, None] * sk[None, None, :]
    U = -db_r[:, None, None] * sk[None, None, :] * np.ones((1, 3, 1))
    L = sk[None, :, None] * da_l[:, None, None] * ones[None, None, :]
    return scale[None, :, None] * D, scale[None, :, None] * L, scale[None, :, None] * U


def spatial_jacobian(prob: Problem, v: np.ndarray) -> sp.csr_matrix:
    """dF/dv as a sparse (3 nx) x (3 nx) matrix in (k, j) ordering (index k nx + j)."""
    nx = prob.nx
    D, L, U = spatial_blocks(prob, v)
    rows, cols, vals = [], [], []
    j = np.arange(nx)
    for blk, shift in ((D, 0), (L, -1), (U, 1)):
        jc = (j + shift) % nx
        for k in range(3):
            for m in range(3):
                rows.append(k * nx + j)
                cols.append(m * nx + jc)
                vals.append(blk[:, k, m])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(3 * nx, 3 * nx))


def p2_residual(prob: Problem, u: np.ndarray) -> np.ndarray:
    """A(u) of shape (N_t, 3, N_x) for u of shape (N_t+1, 3, N_x)."""
    nt, ht = prob.nt, prob.ht
    out = np.empty((nt, 3, prob.nx))
    for l in range(nt):
        c0, c1, c2 = time_coeffs(prob.time, l)
        t = c0 * u[l + 1] + c1 * u[l]
        if c2 != 0.0:
            t = t + c2 * u[l - 1]
        out[l] = t / ht + spatial_operator(prob, u[l + 1])
    return out


def p2_jacobian(prob: Problem, u: np.ndarray) -> sp.csr_matrix:
    """dA/dU for the unknown levels U = (u^1..u^{N_t}); rows (l, k, j), columns (m-1, k', j')."""
    nt, n, ht = prob.nt, 3 * prob.nx, prob.ht
    blocks = [[None] * nt for _ in range(nt)]
    eye = sp.identity(n, format="csr")
    for l in range(nt):
        c0, c1, c2 = time_coeffs(prob.time, l)
        blocks[l][l] = (c0 / ht) * eye + spatial_jacobian(prob, u[l + 1])
        if l >= 1:
            blocks[l][l - 1] = (c1 / ht) * eye
        if l >= 2 and c2 != 0.0:
            blocks[l][l - 2] = (c2 / ht) * eye
    return sp.bmat(blocks, format="csr")


def p2_apply_j(prob: Problem, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    return (p2_jacobian(prob, u) @ v.ravel()).reshape(v.shape)


def p2_apply_jt(prob: Problem, u: np.ndarray, phi: np.ndarray) -> np.ndarray:
    return (p2_jacobian(prob, u).T @ phi.ravel()).reshape(phi.shape)


def p2_wnorm(prob: Problem, z: np.ndarray) -> float:
    return wnorm(prob, z)


def p2_newton_march(prob: Problem, u0: np.ndarray, tol: float = 1e-14, max_newton: int = 50) -> np.ndarray:
    """Sequential Newton solve of each implicit step; u0 is the (3, nx) coefficient array."""
    nt, ht = prob.nt, prob.ht
    u = np.empty((nt + 1, 3, prob.nx))
    u[0] = u0
    eye = sp.identity(3 * prob.nx, format="csc")
    for l in range(nt):
        c0, c1, c2 = time_coeffs(prob.time, l)
        known = c1 * u[l] + (c2 * u[l - 1] if c2 != 0.0 else 0.0)
        v = u[l].copy()
        for _ in range(max_newton):
            g = (c0 * v + known) / ht + spatial_operator(prob, v)
            jac = ((c0 / ht) * eye + spatial_jacobian(prob, v)).tocsc()
            dv = spla.spsolve(jac, g.ravel()).reshape(v.shape)
            v -= dv
            if np.max(np.abs(dv)) <= tol * max(1.0, np.max(np.abs(v))):
                break
        u[l + 1] = v
    return u


# ------------------------------------------------------------------ preconditioner
def unit_upwind_blocks(prob: Problem):
    """(G_0, G_-1): blocks of the unit-speed upwind DG operator (the linear flux f(u) = u,
    for which the local Lax-Friedrichs flux is the upwind flux)."""
    lin = Problem(nx=prob.nx, nt=prob.nt, length=prob.length, t_final=prob.t_final, alpha=0.0, beta=1.0,
                  space="dg_p2_llf")
    D, L, _ = spatial_blocks(lin, np.zeros((3, prob.nx)))
    return D[0], L[0]


def symbol(prob: Problem, theta: float) -> np.ndarray:
    g0, gm = unit_upwind_blocks(prob)
    return g0 + gm * np.exp(-1j * theta)


def mode_eig(prob: Problem):
    """Per Fourier mode m = 0..nx-1: (lambda_m [3], Q_m [3x3]) of c^2 G(theta_m) G(theta_m)^*."""
    lam = np.empty((prob.nx, 3))
    Q = np.empty((prob.nx, 3, 3), dtype=np.complex128)
    for m in range(prob.nx):
        g = symbol(prob, 2.0 * np.pi * m / prob.nx)
        w, q = np.linalg.eigh(prob.precond_c ** 2 * (g @ g.conj().T))
        lam[m], Q[m] = w, q
    return lam, Q


def p2_kd_solve(prob: Problem, r: np.ndarray) -> np.ndarray:
    """s = K_d^{-1} r for r of shape (N_t, 3, N_x): FFT over cells, per-mode eigenbasis of
    c^2 G G^*, one banded (here dense) solve along t per eigen-branch, back."""
    b = time_matrix(prob)
    kt = b @ b.T
    R = np.fft.fft(r, axis=-1)                            # (nt, 3, nx)
    lam, Q = mode_eig(prob)
    S = np.empty_like(R)
    I = np.eye(prob.nt)
    for m in range(prob.nx):
        w = R[:, :, m] @ Q[m].conj()                      # rows: Q^* rhat_l
        z = np.empty_like(w)
        for br in range(3):
            z[:, br] = sla.solve(kt + lam[m, br] * I, w[:, br], assume_a="pos")
        S[:, :, m] = z @ Q[m].T                           # rows: Q z_l
    return np.real(np.fft.ifft(S, axis=-1))


def p2_kd_dense(prob: Problem) -> np.ndarray:
    """K_d assembled densely (tiny grids only), rows/columns in (l, k, j) ordering."""
    nx = prob.nx
    g0, gm = unit_upwind_blocks(prob)
    G = np.zeros((3 * nx, 3 * nx))
    for j in range(nx):
        for k in range(3):
            for m in range(3):
                G[k * nx + j, m * nx + j] += g0[k, m]
                G[k * nx + j, m * nx + (j - 1) % nx] += gm[k, m]
    b = time_matrix(prob)
    return np.kron(b @ b.T, np.eye(3 * nx)) + np.kron(np.eye(prob.nt), prob.precond_c ** 2 * (G @ G.T))


def default_speed(prob: Problem, u0: np.ndarray) -> float:
    """max |f'(u0_h)| over the cell-edge traces of the projected initial data."""
    a, b = traces(np.asarray(u0))
    return float(max(np.max(np.abs(prob.fp(a))), np.max(np.abs(prob.fp(b)))))
