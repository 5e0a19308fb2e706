"""DG P1 nodal discretisation with the upwind flux (Sections 3.2.2 and 3.2.3) -- oracle,
test infrastructure only.

The paper's own DG example.  On N_x uniform periodic cells I_j = [j h, (j+1) h]
(the paper's x_{1/2} = 0 convention, 0-based), u_h is linear in each cell and
is stored by its values at the two points x_c -+ h/4 (x_c the cell centre):

    xi = 2 (x - x_c) / h,  nodes xi = -1/2 and xi = +1/2,
    basis phi_1 = 1/2 - xi,  phi_2 = 1/2 + xi,  u_h = v_j1 phi_1 + v_j2 phi_2 on I_j.

The weak form on each cell with test function phi_k,

    M dv_j/dt = int_{I_j} f(u_h) phi_k' dx - fhat_{j+1/2} phi_k(x_{j+1/2}^-) + fhat_{j-1/2} phi_k(x_{j-1/2}^+),

M = h [[7/12, -1/12], [-1/12, 7/12]] the mass matrix, fhat the upwind flux
f(u^-) (the paper's choice for f' >= 0), the volume integral exact by the
2-point Gauss rule (f quadratic).  Written dv/dt + F(v) = 0; the implicit
scheme in time is that of Section 3.1 coefficient-wise:
A^l = (c0 v^{l+1} + c1 v^l + c2 v^{l-1}) / h_t + F(v^{l+1}).  For the linear flux
this is dv_j/dt = A_1 v_j + A_2 v_{j-1}; for f = alpha u^2 + beta u it is the
quadratic-form system with the matrices C_1..C_9 of the appendix, both printed
in the paper and reproduced by the tests.

Arrays: u [N_t+1][2][N_x] (two nodal planes), residual and phi [N_t][2][N_x];
norm of a space-time array sqrt(h_t h_x sum z^2), as for finite differences.
Preconditioner: the Gram reading of the finite-difference case with the
spatial part c^2 G G^T, G the unit-speed upwind P1 operator (blocks G_0 on the
diagonal, G_-1 below it); per Fourier mode over the cells the two planes
couple through the 2x2 Hermitian c^2 G(theta) G(theta)^*.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fd import time_matrix, wnorm
from .problem import Problem, time_coeffs

NODES = np.array([-0.5, 0.5])                    # nodal points in xi
GAUSS_X = np.array([-1.0, 1.0]) / np.sqrt(3.0)    # 2-point Gauss on [-1, 1], weights 1
MASS_UNIT = np.array([[7.0, -1.0], [-1.0, 7.0]]) / 12.0   # M / h


def basis(xi):
    """(phi_1, phi_2) at xi, stacked on the first axis."""
    xi = np.asarray(xi, dtype=np.float64)
    return np.stack([0.5 - xi, 0.5 + xi])


DBASIS = np.array([-1.0, 1.0])                   # d phi_k / d xi


def mass_unit() -> np.ndarray:
    """int_{-1}^{1} phi_k phi_m dxi / 2 by the 2-point Gauss rule (exact for the product of two
    linear functions): the mass matrix divided by h."""
    P = basis(GAUSS_X)
    return 0.5 * P @ P.T


def interpolate(fn, nx: int, length: float = 1.0) -> np.ndarray:
    """Nodal values (fn(x_c - h/4), fn(x_c + h/4)) per cell: shape (2, nx)."""
    h = length / nx
    xc = (np.arange(nx) + 0.5) * h
    return np.stack([fn(xc - 0.25 * h), fn(xc + 0.25 * h)])


def node_x(nx: int, length: float = 1.0) -> np.ndarray:
    h = length / nx
    xc = (np.arange(nx) + 0.5) * h
    return np.stack([xc - 0.25 * h, xc + 0.25 * h])


def traces(v: np.ndarray):
    """(a, b): right-edge values a_j = u_h(x_{j+1/2}^-) and left-edge values b_j = u_h(x_{j-1/2}^+)."""
    P1, P_1 = basis(1.0), basis(-1.0)
    a = P1[0] * v[0] + P1[1] * v[1]
    b = P_1[0] * v[0] + P_1[1] * v[1]
    return a, b


def spatial_operator(prob: Problem, v: np.ndarray) -> np.ndarray:
    """F(v), shape (2, nx): minus M^{-1} times the weak-form right-hand side with the upwind flux."""
    h = prob.hx
    a, _ = traces(v)
    fhat_r = prob.f(a)                   # fhat_{j+1/2} = f(u^-) from cell j
    fhat_l = np.roll(fhat_r, 1)          # fhat_{j-1/2} from cell j-1
    P = basis(GAUSS_X)                    # (2 basis, 2 points)
    uq = P.T @ v                          # u_h at the Gauss points: (2 points, nx)
    vol = DBASIS[:, None] * np.sum(prob.f(uq), axis=0)[None, :]   # int f(u_h) dphi_k/dxi dxi
    P1, P_1 = basis(1.0), basis(-1.0)
    rhs = vol - fhat_r[None, :] * P1[:, None] + fhat_l[None, :] * P_1[:, None]
    minv = np.linalg.inv(h * mass_unit())
    return -(minv @ rhs)


def spatial_blocks(prob: Problem, v: np.ndarray):
    """2x2 blocks of dF/dv per cell: (D, L) with F_j depending on v_j (D_j) and v_{j-1} (L_j).
    Arrays of shape (nx, 2, 2)."""
    h, nx = prob.hx, prob.nx
    a, _ = traces(v)
    P = basis(GAUSS_X)
    uq = P.T @ v
    P1, P_1 = basis(1.0), basis(-1.0)
    minv = np.linalg.inv(h * mass_unit())
    # d vol_k / d v_m = dphi_k sum_q f'(u_q) phi_m(x_q), per cell j: (nx, k, m)
    dvol = DBASIS[None, :, None] * (P @ prob.fp(uq)).T[:, None, :]
    # d(fhat_{j+1/2} phi_k(1)) / d v_j  and  d(fhat_{j-1/2} phi_k(-1)) / d v_{j-1}
    dflux_r = prob.fp(a)[:, None, None] * np.outer(P1, P1)[None]
    dflux_l = prob.fp(np.roll(a, 1))[:, None, None] * np.outer(P_1, P1)[None]
    D = -np.einsum("kl,jlm->jkm", minv, dvol - dflux_r)
    L = -np.einsum("kl,jlm->jkm", minv, dflux_l)
    return D, L


def spatial_jacobian(prob: Problem, v: np.ndarray) -> sp.csr_matrix:
    """dF/dv as a sparse (2 nx) x (2 nx) matrix in (k, j) ordering (index k nx + j)."""
    nx = prob.nx
    D, L = spatial_blocks(prob, v)
    j = np.arange(nx)
    rows, cols, vals = [], [], []
    for k in range(2):
        for m in range(2):
            rows += [k * nx + j, k * nx + j]
            cols += [m * nx + j, m * nx + (j - 1) % nx]
            vals += [D[:, k, m], L[:, k, m]]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(2 * nx, 2 * nx))


def p1_residual(prob: Problem, u: np.ndarray) -> np.ndarray:
    """A(u) of shape (N_t, 2, N_x) for u of shape (N_t+1, 2, N_x)."""
    nt, ht = prob.nt, prob.ht
    out = np.empty((nt, 2, prob.nx))
    for l in range(nt):
        c0, c1, c2 = time_coeffs(prob.time, l)
        t = c0 * u[l + 1] + c1 * u[l]
        if c2 != 0.0:
            t = t + c2 * u[l - 1]
        out[l] = t / ht + spatial_operator(prob, u[l + 1])
    return out


def p1_jacobian(prob: Problem, u: np.ndarray) -> sp.csr_matrix:
    """dA/dU for the unknown levels U = (u^1..u^{N_t}); rows (l, k, j)."""
    nt, n, ht = prob.nt, 2 * prob.nx, prob.ht
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


def p1_apply_j(prob: Problem, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    return (p1_jacobian(prob, u) @ v.ravel()).reshape(v.shape)


def p1_apply_jt(prob: Problem, u: np.ndarray, phi: np.ndarray) -> np.ndarray:
    return (p1_jacobian(prob, u).T @ phi.ravel()).reshape(phi.shape)


def p1_wnorm(prob: Problem, z: np.ndarray) -> float:
    return wnorm(prob, z)


def p1_newton_march(prob: Problem, u0: np.ndarray, tol: float = 1e-14, max_newton: int = 50) -> np.ndarray:
    """Sequential Newton solve of each implicit step; u0 is the (2, nx) nodal array."""
    nt, ht = prob.nt, prob.ht
    u = np.empty((nt + 1, 2, prob.nx))
    u[0] = u0
    eye = sp.identity(2 * prob.nx, format="csc")
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


def space_time_error(prob: Problem, u: np.ndarray, exact) -> float:
    """sqrt(h_t h_x sum_{l, j, k} (u^l_jk - exact(x_jk, t_l))^2) over all levels: the discrete
    L^2(Omega x [0, T]) error with each nodal value weighted h_t h_x (the norm of the residuals)."""
    xs = node_x(prob.nx, prob.length)
    err = 0.0
    for l in range(prob.nt + 1):
        err += np.sum((u[l] - exact(xs, l * prob.ht)) ** 2)
    return float(np.sqrt(prob.ht * prob.hx * err))


# ------------------------------------------------------------------ preconditioner
def unit_upwind_blocks(prob: Problem):
    """(G_0, G_-1): blocks of the unit-speed upwind P1 operator (f(u) = u)."""
    lin = Problem(nx=prob.nx, nt=prob.nt, length=prob.length, t_final=prob.t_final, alpha=0.0, beta=1.0,
                  space="dg_p1_upwind")
    D, L = spatial_blocks(lin, np.zeros((2, prob.nx)))
    return D[0], L[0]


def symbol(prob: Problem, theta: float, blocks=None) -> np.ndarray:
    g0, gm = unit_upwind_blocks(prob) if blocks is None else blocks
    return g0 + gm * np.exp(-1j * theta)


def mode_eig(prob: Problem):
    """Per Fourier mode m = 0..nx-1: (lambda_m [2], Q_m [2x2]) of c^2 G(theta_m) G(theta_m)^*."""
    lam = np.empty((prob.nx, 2))
    Q = np.empty((prob.nx, 2, 2), dtype=np.complex128)
    blocks = unit_upwind_blocks(prob)
    for m in range(prob.nx):
        g = symbol(prob, 2.0 * np.pi * m / prob.nx, blocks)
        w, q = np.linalg.eigh(prob.precond_c ** 2 * (g @ g.conj().T))
        lam[m], Q[m] = w, q
    return lam, Q


def p1_kd_solve(prob: Problem, r: np.ndarray) -> np.ndarray:
    """s = K_d^{-1} r for r of shape (N_t, 2, N_x): FFT over cells, per-mode eigenbasis of
    c^2 G G^*, one (here dense) solve along t per eigen-branch, back."""
    b = time_matrix(prob)
    kt = b @ b.T
    R = np.fft.fft(r, axis=-1)
    lam, Q = mode_eig(prob)
    S = np.empty_like(R)
    I = np.eye(prob.nt)
    for m in range(prob.nx):
        w = R[:, :, m] @ Q[m].conj()
        z = np.empty_like(w)
        for br in range(2):
            z[:, br] = sla.solve(kt + lam[m, br] * I, w[:, br], assume_a="pos")
        S[:, :, m] = z @ Q[m].T
    return np.real(np.fft.ifft(S, axis=-1))


def p1_kd_dense(prob: Problem) -> np.ndarray:
    """K_d assembled densely (tiny grids only), rows/columns in (l, k, j) ordering."""
    nx = prob.nx
    g0, gm = unit_upwind_blocks(prob)
    G = np.zeros((2 * nx, 2 * nx))
    for j in range(nx):
        for k in range(2):
            for m in range(2):
                G[k * nx + j, m * nx + j] += g0[k, m]
                G[k * nx + j, m * nx + (j - 1) % nx] += gm[k, m]
    b = time_matrix(prob)
    return np.kron(b @ b.T, np.eye(2 * nx)) + np.kron(np.eye(prob.nt), prob.precond_c ** 2 * (G @ G.T))


def default_speed(prob: Problem, u0: np.ndarray) -> float:
    """max |f'| over the nodal values and the cell-edge traces of the initial data."""
    u0 = np.asarray(u0)
    a, b = traces(u0)
    return float(max(np.max(np.abs(prob.fp(u0))), np.max(np.abs(prob.fp(a))), np.max(np.abs(prob.fp(b)))))
