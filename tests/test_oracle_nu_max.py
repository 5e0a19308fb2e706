"""Pins of the oracle's step-size estimates (CPU only).

Proposition 2.1 (Section 2.3) asks for sigma tau nu < 1 for every eigenvalue nu
of J^T K_d^{-1} J; the oracle estimates the largest one by power iteration
(``oracle.pdhg.nu_max``, and ``oracle.onestep.auto_steps`` over the one-level
step operators of Algorithm 3).  Here those estimates are compared with the
largest eigenvalue of the same matrix assembled densely on tiny grids and
handed to LAPACK: J as an explicit matrix, K_d as a dense matrix assembled
independently of the FFT solve (Kronecker products for finite differences, the
block-circulant DG forms), and for Algorithm 3's step the one-level
K_l = (c0/h_t)^2 I + c^2 L_x + ghat^2 L_x^2 written out here from its
definition.

The power iteration returns a Rayleigh quotient of a symmetric positive
semi-definite matrix, so it can only under-estimate: it must lie in
[0.99, 1 + 1e-12] x lambda_max after the solver's 200 iterations, and agree
to 1e-8 after 3000.
"""
import numpy as np
import pytest

import synthetic as syn
from oracle import dg, dg1, fd, onestep, pdhg, precond
from oracle.problem import Problem, default_constants


def _lam_max(J, K):
    M = J.T @ np.linalg.solve(K, J)
    return float(np.max(np.linalg.eigvalsh(0.5 * (M + M.T))))


def _check(est200, est3000, lam):
    assert est200 <= lam * (1 + 1e-12)
    assert est200 >= 0.99 * lam
    assert abs(est3000 - lam) <= 1e-8 * lam


@pytest.mark.parametrize("space,time,gamma,ghat", [
    ("fd_lf", "bdf2", 0.0, 0.0), ("fd_lf", "be", 1e-3, 1e-3), ("fd_upwind", "be", 0.0, 0.0),
    ("fd_upwind", "bdf2", 0.0, 0.2)])
def test_nu_max_finite_differences(space, time, gamma, ghat):
    nx, nt = 16, 6
    u0 = syn.fourier_u0(1, nx)
    prob = default_constants(Problem(nx=nx, nt=nt, t_final=0.3, alpha=0.5, beta=0.0, gamma=gamma, time=time,
                                     space=space, precond_gamma_hat=ghat), u0)
    u = np.tile(u0, (nt + 1, 1))
    lam = _lam_max(fd.jacobian(prob, u).toarray(), precond.kd_dense(prob))
    _check(pdhg.nu_max(prob, u), pdhg.nu_max(prob, u, iters=3000), lam)
    t, _, nm = pdhg.auto_steps(prob, u0)
    assert nm == pytest.approx(pdhg.nu_max(prob, u), rel=1e-14)
    assert t * t * lam <= 0.95 * (1 + 1e-9) / 0.99


def test_nu_max_at_a_general_iterate():
    """Away from u^l = u0: a random space-time field (the linearisation point of a later iterate)."""
    nx, nt = 12, 5
    u0 = syn.fourier_u0(2, nx)
    prob = default_constants(Problem(nx=nx, nt=nt, t_final=0.4, alpha=0.5, beta=0.0, time="bdf2",
                                     space="fd_lf"), u0)
    u = np.tile(u0, (nt + 1, 1)) + 0.2 * np.random.default_rng(5).standard_normal((nt + 1, nx))
    u[0] = u0
    lam = _lam_max(fd.jacobian(prob, u).toarray(), precond.kd_dense(prob))
    _check(pdhg.nu_max(prob, u), pdhg.nu_max(prob, u, iters=3000), lam)


def _dense_from_apply(apply, shape):
    n = int(np.prod(shape))
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        cols.append(apply(e.reshape(shape)).ravel())
    return np.array(cols).T


def test_nu_max_dg_p2():
    nx, nt = 4, 3
    u0 = dg.p2_project(lambda x: syn.fourier_u0_at(0, x), nx)
    prob = default_constants(Problem(nx=nx, nt=nt, t_final=0.15, alpha=0.5, beta=0.0, time="be",
                                     space="dg_p2_llf"), u0)
    u = np.broadcast_to(u0, (nt + 1,) + u0.shape).copy()
    J = _dense_from_apply(lambda v: dg.p2_apply_j(prob, u, v), (nt, 3, nx))
    lam = _lam_max(J, dg.p2_kd_dense(prob))
    _check(pdhg.nu_max(prob, u), pdhg.nu_max(prob, u, iters=3000), lam)


def test_nu_max_dg_p1():
    nx, nt = 6, 3
    u0 = dg1.interpolate(lambda x: syn.fourier_u0_at(0, x), nx)
    prob = default_constants(Problem(nx=nx, nt=nt, t_final=0.2, alpha=0.0, beta=1.0, time="bdf2",
                                     space="dg_p1_upwind"), u0)
    u = np.broadcast_to(u0, (nt + 1,) + u0.shape).copy()
    J = dg1.p1_jacobian(prob, u).toarray()
    lam = _lam_max(J, dg1.p1_kd_dense(prob))
    _check(pdhg.nu_max(prob, u), pdhg.nu_max(prob, u, iters=3000), lam)


def _step_k_dense(prob, c0):
    """K_l = (c0/h_t)^2 I + c^2 L_x + ghat^2 L_x^2, L_x the periodic (-1, 2, -1)/h_x^2 Laplacian."""
    n = prob.nx
    L = np.zeros((n, n))
    for j in range(n):
        L[j, j] = 2.0
        L[j, (j - 1) % n] = -1.0
        L[j, (j + 1) % n] = -1.0
    L /= prob.hx ** 2
    return (c0 / prob.ht) ** 2 * np.eye(n) + prob.precond_c ** 2 * L + prob.precond_gamma_hat ** 2 * (L @ L)


@pytest.mark.parametrize("time", ["be", "bdf2"])
def test_onestep_auto_steps(time):
    """Algorithm 3's step sizes: the largest eigenvalue of J_l^T K_l^{-1} J_l over the step operators
    (c0 = 1, and 3/2 for BDF2), J_l = (c0/h_t) I + dF(u0)."""
    nx, nt = 16, 8
    u0 = syn.fourier_u0(3, nx)
    prob = default_constants(Problem(nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.0, gamma=1e-3, time=time,
                                     space="fd_lf", precond_gamma_hat=1e-3), u0)
    lam = 0.0
    for c0 in ([1.0, 1.5] if time == "bdf2" else [1.0]):
        # dF(u0) as the N_t = 1 Jacobian minus its time part 1/h_t
        q = prob.with_(nt=1, time="be")
        JF = fd.jacobian(q, np.stack([u0, u0])).toarray() - np.eye(nx) / q.ht
        Jl = (c0 / prob.ht) * np.eye(nx) + JF
        lam = max(lam, _lam_max(Jl, _step_k_dense(prob, c0)))
    t, t2, nm = onestep.auto_steps(prob, u0)
    assert nm <= lam * (1 + 1e-12) and nm >= 0.99 * lam
    _, _, nm_tight = onestep.auto_steps(prob, u0, iters=3000)
    assert abs(nm_tight - lam) <= 1e-8 * lam
    assert t == t2 == pytest.approx(np.sqrt(0.95 / nm))
