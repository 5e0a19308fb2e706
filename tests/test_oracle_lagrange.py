"""Pins of the multiplier form of Algorithm 1 (u^0 free, lambda imposing u^0 = u0; Section 3.3) in the
oracle (CPU only)."""
import json
import os

import numpy as np
import pytest

import synthetic as syn
from oracle import closed_form, fd, lagrange, newton, pdhg
from oracle.problem import Problem, default_constants

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("tm", ["be", "bdf2"])
def test_steps_are_the_gradients_of_the_printed_lagrangian(tm):
    """The u^0 step direction h_t J_0^T phi + lambda is (1/h_x) dL/du^0 and the u^l step direction
    J^T phi is (1/(h_t h_x)) dL/du^l, with L as printed in Section 3.3; central differences of L."""
    nx, nt = 16, 5
    u0 = syn.fourier_u0(3, nx)
    prob = default_constants(Problem(nx=nx, nt=nt, t_final=0.3, alpha=0.5, beta=0.0, space="fd_lf", time=tm), u0)
    rng = np.random.default_rng(1)
    u = np.tile(u0, (nt + 1, 1)) + 0.1 * rng.standard_normal((nt + 1, nx))
    phi = rng.standard_normal((nt, nx))
    lam = rng.standard_normal(nx)
    g0 = lagrange.j0t(prob, phi) + lam
    gl = fd.apply_jt(prob, u, phi)
    h = 1e-6
    for j in (0, 5, 11):
        up, um = u.copy(), u.copy()
        up[0, j] += h
        um[0, j] -= h
        d = (lagrange.lagrangian(prob, up, phi, lam, u0) - lagrange.lagrangian(prob, um, phi, lam, u0)) / (2 * h)
        assert d / prob.hx == pytest.approx(g0[j], rel=1e-7, abs=1e-8)
        for l in (1, nt):
            up, um = u.copy(), u.copy()
            up[l, j] += h
            um[l, j] -= h
            d = (lagrange.lagrangian(prob, up, phi, lam, u0) - lagrange.lagrangian(prob, um, phi, lam, u0)) / (2 * h)
            assert d / (prob.ht * prob.hx) == pytest.approx(gl[l - 1, j], rel=1e-7, abs=1e-6)
    # and the lambda step is (1/h_x) dL/dlambda = u^0 - u0
    dl = np.zeros(nx)
    dl[4] = h
    d = (lagrange.lagrangian(prob, u, phi, lam + dl, u0) - lagrange.lagrangian(prob, u, phi, lam - dl, u0)) / (2 * h)
    assert d / prob.hx == pytest.approx(u[0, 4] - u0[4], rel=1e-7, abs=1e-12)


def test_frozen_multiplier_block_is_algorithm_1_with_fixed_initial_level():
    """tau_u0 = 0 and tau_lam = 0 leave u^0 = u0 and lambda = 0: the iterates are those of pdhg.run."""
    u0 = syn.fourier_u0(1, 32)
    prob = default_constants(Problem(nx=32, nt=9, t_final=0.5, alpha=0.5, beta=0.0, space="fd_lf", time="bdf2"), u0)
    a = lagrange.run(prob, u0, 0.6, 0.6, 0.0, eps=0.0, max_iter=25, tau_u0=0.0)
    b = pdhg.run(prob, u0, 0.6, 0.6, eps=0.0, max_iter=25)
    assert np.array_equal(a.u, b.u) and np.array_equal(a.phi, b.phi)


@pytest.mark.parametrize("tm", ["be", "bdf2"])
def test_limit_is_the_implicit_scheme_with_the_given_initial_data(tm):
    """Burgers LF 64 x 16: the saddle point has u^0 = u0, A(u) = 0, phi = 0 and lambda = 0, so the limit is
    the Newton march of the scheme."""
    u0 = syn.fourier_u0(0, 64)
    prob = default_constants(Problem(nx=64, nt=16, t_final=0.5, alpha=0.5, beta=0.0, space="fd_lf", time=tm), u0)
    tu, tp, _ = pdhg.auto_steps(prob, u0)
    res = lagrange.run(prob, u0, tu, tp, 0.99, eps=1e-9, max_iter=20000)
    assert res.converged
    nw = newton.march(prob, u0)
    assert np.max(np.abs(res.u - nw)) < 1e-8
    assert np.max(np.abs(res.u[0] - u0)) < 1e-8
    assert np.max(np.abs(res.phi)) < 1e-8 and np.max(np.abs(res.lam)) < 1e-7


def test_advection_closed_form():
    prob = default_constants(Problem(nx=64, nt=32, t_final=2.0, alpha=0.0, beta=1.0, space="fd_upwind",
                                     time="be"), syn.sine_u0(64))
    res = lagrange.run(prob, syn.sine_u0(64), 0.7, 0.7, 0.99, eps=1e-10, max_iter=5000)
    assert res.converged
    assert np.max(np.abs(res.u - closed_form.advection_sine_solution(64, 32, 4.0))) < 1e-10


@pytest.mark.parametrize("case", [0, 1, 2])
def test_table1_with_the_multiplier(case):
    """Table 1's heat runs with the multiplier form as printed in Algorithm 1 (tau = (0.8, 0.8, 0.99)):
    iterations to 1e-6 and 1e-10 within +15 % of the printed counts."""
    with open(os.path.join(GOLDEN, "table1_heat_iterations.json")) as fh:
        t1 = json.load(fh)
    nx, nt = t1["grids_nx_nt"][case]
    prob = Problem(nx=nx, nt=nt, t_final=0.1, alpha=0.0, beta=0.0, space="heat_var", time="be", precond_c=0.0,
                   precond_gamma_hat=0.6, gamma_fn=syn.heat_gamma_at)
    res = lagrange.run(prob, syn.gaussian_bump_u0(nx), 0.8, 0.8, 0.99, eps=1e-10, max_iter=400, record=True)
    n6 = next(n for n, rp, rd, _ in res.history if max(rp, rd) <= 1e-6)
    assert res.converged
    for got, want in ((n6, t1["iterations_eps_1e-6"][case]), (res.iters, t1["iterations_eps_1e-10"][case])):
        assert want * 0.97 <= got <= want * 1.15, (nx, nt, got, want)
