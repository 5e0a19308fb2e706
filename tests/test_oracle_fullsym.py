"""Pins of the full-symbol preconditioner (oracle/precond.py): K_full = J_c J_c^T with J_c the scheme's
Jacobian for the linear flux f = c u, solved per FFT mode by two triangular substitutions."""
import numpy as np
import pytest

import synthetic as syn
from oracle import fd
from oracle import newton as onewton
from oracle import onestep as oos
from oracle import pdhg as opdhg
from oracle.precond import kd_full_solve
from oracle.problem import Problem, default_constants


def _linear_jacobian(p):
    """J_c assembled by the finite-difference oracle for the linear flux c u (any u: the flux is linear)."""
    lin = p.with_(alpha=0.0, beta=p.precond_c, gamma=p.precond_gamma_hat)
    return fd.jacobian(lin, np.zeros((p.nt + 1, p.nx))).toarray()


@pytest.mark.parametrize("space,time,ghat", [("fd_lf", "be", 0.0), ("fd_lf", "bdf2", 0.0), ("fd_upwind", "bdf2", 0.0),
                                             ("fd_lf", "be", 2e-3)])
def test_solve_against_the_dense_gram_of_the_linear_jacobian(space, time, ghat):
    p = Problem(nx=16, nt=7, t_final=0.3, alpha=0.5, beta=0.0, time=time, space=space, lf_speed=0.8,
                precond_c=0.6, precond_gamma_hat=ghat, precond_kind="full")
    J = _linear_jacobian(p)
    r = np.random.default_rng(1).standard_normal((7, 16))
    ref = np.linalg.solve(J @ J.T, r.ravel()).reshape(r.shape)
    np.testing.assert_allclose(kd_full_solve(p, r), ref, rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("time", ["be", "bdf2"])
def test_linear_transport_is_preconditioned_exactly(time):
    """For linear upwind transport with c = a, J^T K_full^{-1} J = I: every eigenvalue nu is 1."""
    p = Problem(nx=32, nt=8, t_final=0.5, alpha=0.0, beta=1.3, time=time, space="fd_upwind", precond_c=1.3,
                precond_kind="full")
    J = fd.jacobian(p, np.zeros((9, 32)))
    v = np.random.default_rng(2).standard_normal((8, 32))
    w = (J @ v.ravel()).reshape(v.shape)
    back = (J.T @ kd_full_solve(p, w).ravel()).reshape(v.shape)
    np.testing.assert_allclose(back, v, rtol=1e-11, atol=1e-11)


def test_burgers_converges_to_the_newton_march_in_fewer_iterations():
    u0 = syn.fourier_u0(0, 64)
    base = Problem(nx=64, nt=16, t_final=0.5, alpha=0.5, beta=0.0, time="bdf2", space="fd_lf")
    runs = {}
    for kind in ("gram", "full"):
        p = default_constants(base.with_(precond_kind=kind), u0)
        tu, tp, _ = opdhg.auto_steps(p, u0)
        res = opdhg.run(p, u0, tu, tp, eps=1e-8, max_iter=5000)
        assert res.converged
        np.testing.assert_allclose(res.u, onewton.march(p, u0), atol=2e-8)
        runs[kind] = res.iters
    assert runs["full"] * 4 < runs["gram"], runs


def test_one_step_full_symbol_is_exact_for_linear_transport():
    """One level: J_l^T K_l^{-1} J_l = I with K_l = |c0/h_t + g_k|^2 per mode, so a step with
    sigma tau = 0.95 contracts by sqrt(0.05) per iteration."""
    p = Problem(nx=32, nt=4, t_final=0.2, alpha=0.0, beta=1.0, time="be", space="fd_upwind", precond_c=1.0,
                precond_kind="full")
    u0 = syn.fourier_u0(0, 32)
    hist = []
    t = np.sqrt(0.95)
    oos.solve_step(p, 0, u0, None, t, t, eps=0.0, max_iter=40, hist=hist)
    h = np.array(hist)
    r = np.maximum(h[:, 1], h[:, 2])
    win = (r < 1e-2) & (r > 1e-12)
    slope = np.polyfit(h[win, 0], np.log(r[win]), 1)[0]
    assert abs(np.exp(slope) - np.sqrt(0.05)) < 0.02
