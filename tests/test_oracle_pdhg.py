"""Pins of the oracle's preconditioner, primal-dual loop and adjoint (CPU only)."""
import json
import os

import numpy as np
import pytest

import synthetic as syn
from oracle import adjoint, closed_form, fd, newton, pdhg, precond
from oracle.problem import Problem, default_constants

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ preconditioner
@pytest.mark.parametrize("tm", ["be", "bdf2"])
@pytest.mark.parametrize("c,g", [(0.0, 0.6), (1.3, 0.0), (0.7, 0.05)])
def test_kd_solve_matches_dense_kronecker(tm, c, g):
    """FFT + banded solves equal a dense solve of the Kronecker-assembled K_d."""
    prob = Problem(nx=8, nt=6, t_final=0.3, time=tm, precond_c=c, precond_gamma_hat=g)
    r = np.random.default_rng(0).standard_normal((prob.nt, prob.nx))
    s = precond.kd_solve(prob, r)
    dense = np.linalg.solve(precond.kd_dense(prob), r.ravel()).reshape(r.shape)
    assert np.max(np.abs(s - dense)) <= 1e-11 * np.max(np.abs(dense))
    assert np.max(np.abs(precond.kd_apply(prob, s) - r)) <= 1e-9 * np.max(np.abs(r))


def test_time_gram_backward_euler_form():
    """BE: B_t B_t^T = tridiag(-1; 1, 2, ..., 2; -1)/h_t^2 (Neumann at l = 0, phi^{N_t} = 0)."""
    prob = Problem(nx=4, nt=7, t_final=0.7, time="be")
    kt = precond.time_gram(prob) * prob.ht ** 2
    expect = 2 * np.eye(7) - np.eye(7, k=1) - np.eye(7, k=-1)
    expect[0, 0] = 1.0
    assert np.allclose(kt, expect, atol=1e-12)


# ------------------------------------------------------------------ Table 1
def _table1():
    with open(os.path.join(GOLDEN, "table1_heat_iterations.json")) as fh:
        return json.load(fh)


def _heat(nx, nt):
    return Problem(nx=nx, nt=nt, t_final=0.1, alpha=0.0, beta=0.0, space="heat_var", time="be",
                   precond_c=0.0, precond_gamma_hat=0.6, gamma_fn=syn.heat_gamma_at)


@pytest.mark.parametrize("case", [0, 1, 2, 3, 4])
def test_table1_heat_iteration_counts(case):
    """Iterations to eps = 1e-6 and 1e-10 within +15 % of Table 1, and grid independent."""
    t1 = _table1()
    nx, nt = t1["grids_nx_nt"][case]
    prob = _heat(nx, nt)
    assert prob.ht / prob.hx ** 2 == pytest.approx(eval(t1["mesh_ratio_ht_over_hx2"][case]))
    res = pdhg.run(prob, syn.gaussian_bump_u0(nx), 0.8, 0.8, eps=1e-10, max_iter=400, record=True)
    n6 = next(n for n, rp, rd in res.history if max(rp, rd) <= 1e-6)
    n10 = res.iters
    assert res.converged
    for got, want in ((n6, t1["iterations_eps_1e-6"][case]), (n10, t1["iterations_eps_1e-10"][case])):
        assert want * 0.97 <= got <= want * 1.15, (nx, nt, got, want)


# ------------------------------------------------------------------ linear advection
def _advection():
    prob = Problem(nx=64, nt=32, t_final=2.0, alpha=0.0, beta=1.0, space="fd_upwind", time="be")
    return default_constants(prob, syn.sine_u0(64))


def test_pdhg_advection_reaches_closed_form():
    """PDHG to 1e-10 on the CFL-4 advection problem reproduces the BE-upwind closed form."""
    prob = _advection()
    assert prob.precond_c == pytest.approx(1.0)
    res = pdhg.run(prob, syn.sine_u0(64), 0.7, 0.7, eps=1e-10, max_iter=3000)
    assert res.converged
    cf = closed_form.advection_sine_solution(64, 32, 4.0)
    assert np.max(np.abs(res.u - cf)) < 1e-10
    assert np.max(np.abs(res.phi)) < 1e-9


def test_proposition_2_1_convergence_rate():
    """Linear case: the slowest error component contracts by sqrt(1 - s t nu_min) per
    iteration (Proposition 2.1), nu_min the smallest eigenvalue of J^T K_d^{-1} J."""
    prob = Problem(nx=16, nt=8, t_final=0.5, alpha=0.0, beta=1.0, space="fd_upwind", time="be",
                   precond_c=1.0)
    u0 = syn.sine_u0(16)
    u = np.tile(u0, (prob.nt + 1, 1))
    J = fd.jacobian(prob, u).toarray()
    M = J.T @ np.linalg.solve(precond.kd_dense(prob), J)
    nu = np.linalg.eigvalsh(0.5 * (M + M.T))
    st = 0.5
    assert st * nu.max() < 1.0
    rate = np.sqrt(1.0 - st * nu.min())
    res = pdhg.run(prob, u0, np.sqrt(st), np.sqrt(st), eps=0.0, max_iter=400, record=True)
    h = np.array(res.history)
    r = np.maximum(h[:, 1], h[:, 2])
    # complex eigenvalue pairs make the decay oscillate: fit the slope of log r by
    # least squares over the geometric phase (above the rounding floor)
    win = (r < 1e-3) & (r > 1e-11)
    slope = np.polyfit(h[win, 0], np.log(r[win]), 1)[0]
    assert abs(np.exp(slope) - rate) < 0.01, (np.exp(slope), rate)
    assert np.max(np.abs(res.u - newton.march(prob, u0))) < 1e-10


# ------------------------------------------------------------------ Burgers: PDHG vs Newton
@pytest.mark.parametrize("tm,expect_iters", [("be", 458), ("bdf2", 781)])
def test_pdhg_burgers_matches_newton_march(tm, expect_iters):
    """LF Burgers, 64 x 16, T = 0.5: the PDHG saddle point is the implicit-scheme solution,
    phi -> 0 and every level keeps the initial mass."""
    u0 = syn.fourier_u0(0, 64)
    prob = default_constants(Problem(nx=64, nt=16, t_final=0.5, alpha=0.5, beta=0.0, space="fd_lf",
                                     time=tm), u0)
    su, sp_, nm = pdhg.auto_steps(prob, u0)
    assert 1.9 < nm < 2.1
    res = pdhg.run(prob, u0, su, sp_, eps=1e-8, max_iter=5000)
    assert res.converged and abs(res.iters - expect_iters) <= 5
    nw = newton.march(prob, u0)
    assert np.max(np.abs(res.u - nw)) < 2e-8
    assert np.max(np.abs(res.phi)) < 1e-8
    m = fd.mass(prob, res.u)
    assert np.max(np.abs(m - m[0])) < 1e-10


def test_pdhg_warm_start_at_solution_is_fixed_point():
    """Starting at (Newton solution, phi = 0) the iteration does not move."""
    u0 = syn.fourier_u0(2, 32)
    prob = default_constants(Problem(nx=32, nt=8, t_final=0.5, alpha=0.5, beta=0.0, space="fd_lf",
                                     time="bdf2"), u0)
    nw = newton.march(prob, u0)
    res = pdhg.run(prob, u0, 0.6, 0.6, eps=0.0, max_iter=5, u_init=nw, phi_init=np.zeros((8, 32)))
    assert np.max(np.abs(res.u - nw)) < 1e-12


# ------------------------------------------------------------------ adjoint
def test_adjoint_linear_closed_form():
    """Linear advection: dl/du0 = 2 h_x (G^T)^{N_t} (u^{N_t} - target) (Fourier closed form)."""
    prob = Problem(nx=64, nt=32, t_final=2.0, alpha=0.0, beta=1.0, space="fd_upwind", time="be")
    u0, tgt = syn.fourier_u0(0, 64), syn.fourier_u0(1, 64)
    u = newton.march(prob, u0)
    g = adjoint.gradient_u0(prob, u, adjoint.terminal_loss_grad(prob, u, tgt))
    cf = closed_form.advection_terminal_gradient(u0, tgt, 32, 4.0, prob.hx)
    assert np.max(np.abs(g - cf)) <= 1e-12 * np.max(np.abs(cf))


@pytest.mark.parametrize("tm", ["be", "bdf2"])
def test_adjoint_matches_central_differences(tm):
    """Viscous LF Burgers: adjoint gradient against FP64 central differences, h = 1e-6."""
    u0, tgt = syn.fourier_u0(0, 48), syn.fourier_u0(1, 48)
    prob = default_constants(Problem(nx=48, nt=12, t_final=0.5, alpha=0.5, beta=0.0, gamma=1e-3,
                                     space="fd_lf", time=tm), u0)
    u = newton.march(prob, u0)
    g = adjoint.gradient_u0(prob, u, adjoint.terminal_loss_grad(prob, u, tgt))
    for d in syn.unit_directions(2, 48, 4):
        h = 1e-6
        lp = adjoint.terminal_loss(prob, newton.march(prob, u0 + h * d), tgt)
        lm = adjoint.terminal_loss(prob, newton.march(prob, u0 - h * d), tgt)
        assert abs((lp - lm) / (2 * h) - g @ d) <= 1e-8 * max(1e-3, abs(g @ d)) + 1e-10
