"""Pins of the DG P2 / local Lax-Friedrichs oracle (oracle/dg.py) against facts that do not
come from its own code: hand-derived upwind matrices, exact polynomial integration, the
per-mode closed form of the linear scheme, conservation, convergence to the characteristic
solution of Burgers before the shock, central differences and a dense preconditioner."""
import numpy as np
import pytest

import synthetic as syn
from oracle import dg
from oracle import newton as onewton
from oracle import pdhg as opdhg
from oracle.problem import Problem, default_constants


def _prob(**kw):
    base = dict(nx=8, nt=4, t_final=0.2, alpha=0.5, beta=0.0, space="dg_p2_llf", time="be")
    base.update(kw)
    return Problem(**base)


def test_projection_reproduces_piecewise_quadratics():
    rng = np.random.default_rng(0)
    nx, h = 6, 1.0 / 6
    c = rng.standard_normal((3, nx))
    def fn(x):   # the quadratic with Legendre coefficients c in each cell
        j = np.minimum((x / h).astype(int), nx - 1)
        xi = 2.0 * (x - (j + 0.5) * h) / h
        return c[0, j] + c[1, j] * xi + c[2, j] * 0.5 * (3 * xi * xi - 1)
    np.testing.assert_allclose(dg.p2_project(fn, nx), c, atol=1e-13)


def test_projection_keeps_exact_cell_averages_of_a_sine():
    nx = 16
    v = dg.p2_project(lambda x: np.sin(2 * np.pi * x), nx)
    j = np.arange(nx)
    h = 1.0 / nx
    exact = (np.cos(2 * np.pi * j * h) - np.cos(2 * np.pi * (j + 1) * h)) / (2 * np.pi * h)
    np.testing.assert_allclose(v[0], exact, atol=1e-14)


def test_unit_speed_blocks_match_hand_derivation():
    """f(u) = u: fhat = a (upwind), V_j0 = 0, V_j1 = 2 v_j0, V_j2 = 2 v_j1, so
    F_j0 = (a_j - a_{j-1})/h, F_j1 = -(3/h)(2 v_j0 - a_j - a_{j-1}), F_j2 = -(5/h)(2 v_j1 - a_j + a_{j-1})
    with a_j = v_j0 + v_j1 + v_j2."""
    h = 0.125
    prob = _prob(nx=8, alpha=0.0, beta=1.0)
    g0 = np.array([[1, 1, 1], [-3, 3, 3], [5, -5, 5]]) / h
    gm = np.array([[-1, -1, -1], [3, 3, 3], [-5, -5, -5]]) / h
    D, L, U = dg.spatial_blocks(prob, np.random.default_rng(1).standard_normal((3, 8)))
    for j in range(8):
        np.testing.assert_allclose(D[j], g0, rtol=0, atol=1e-12)
        np.testing.assert_allclose(L[j], gm, rtol=0, atol=1e-12)
        np.testing.assert_allclose(U[j], 0.0, atol=1e-12)


def test_volume_term_is_exact_for_burgers():
    """V_jk = int_{-1}^{1} (u_h^2/2) P_k' dxi by exact polynomial integration."""
    P = np.polynomial.Polynomial
    rng = np.random.default_rng(2)
    v = rng.standard_normal((3, 5))
    prob = _prob(nx=5)
    V = dg.volume_term(prob, v)
    basis = [P([1.0]), P([0.0, 1.0]), P([-0.5, 0.0, 1.5])]
    for j in range(5):
        uh = v[0, j] * basis[0] + v[1, j] * basis[1] + v[2, j] * basis[2]
        for k in range(3):
            integrand = 0.5 * uh * uh * basis[k].deriv()
            F = integrand.integ()
            assert V[k, j] == pytest.approx(F(1.0) - F(-1.0), abs=1e-13)


def test_llf_flux_special_cases():
    prob = _prob()
    # equal states: the flux is f(a); same-sign states with a the faster one
    assert dg.llf_flux(prob, 0.7, 0.7) == pytest.approx(prob.f(0.7))
    a, b = 1.0, 0.4
    assert dg.llf_flux(prob, a, b) == pytest.approx(0.5 * (0.5 + 0.08) - 0.5 * 1.0 * (0.4 - 1.0))


@pytest.mark.parametrize("time", ["be", "bdf2"])
def test_jacobian_matches_central_differences(time):
    rng = np.random.default_rng(3)
    prob = _prob(nx=6, nt=3, time=time)
    u = 0.5 + 0.3 * rng.standard_normal((4, 3, 6))
    J = dg.p2_jacobian(prob, u).toarray()
    h = 1e-6
    n = 3 * 3 * 6
    num = np.empty((n, n))
    for c in range(n):
        up, um = u.copy(), u.copy()
        up[1:].reshape(-1)[c] += h
        um[1:].reshape(-1)[c] -= h
        num[:, c] = (dg.p2_residual(prob, up) - dg.p2_residual(prob, um)).ravel() / (2 * h)
    np.testing.assert_allclose(J, num, atol=1e-6 * np.max(np.abs(J)))


def test_transpose_dot_product():
    rng = np.random.default_rng(4)
    prob = _prob(nx=8, nt=3, time="bdf2")
    u = 0.5 + 0.2 * rng.standard_normal((4, 3, 8))
    v, w = rng.standard_normal((3, 3, 8)), rng.standard_normal((3, 3, 8))
    assert np.sum(dg.p2_apply_j(prob, u, v) * w) == pytest.approx(np.sum(v * dg.p2_apply_jt(prob, u, w)), rel=1e-12)


def test_linear_scheme_matches_per_mode_closed_form():
    """f(u) = u, backward Euler: every Fourier mode of the coefficient vector evolves by
    (I + h_t G(theta))^{-1} with G(theta) = G_0 + G_-1 e^{-i theta} from the hand-derived blocks."""
    nx, nt, T = 16, 8, 0.5
    prob = Problem(nx=nx, nt=nt, t_final=T, alpha=0.0, beta=1.0, space="dg_p2_llf", time="be")
    u0 = dg.p2_project(lambda x: np.sin(2 * np.pi * x) + 0.3 * np.cos(6 * np.pi * x), nx)
    u = onewton.march(prob, u0)
    h, ht = 1.0 / nx, T / nt
    g0 = np.array([[1, 1, 1], [-3, 3, 3], [5, -5, 5]]) / h
    gm = np.array([[-1, -1, -1], [3, 3, 3], [-5, -5, -5]]) / h
    U = np.fft.fft(u0, axis=-1)
    for l in range(nt):
        for m in range(nx):
            G = g0 + gm * np.exp(-2j * np.pi * m / nx)
            U[:, m] = np.linalg.solve(np.eye(3) + ht * G, U[:, m])
        np.testing.assert_allclose(np.real(np.fft.ifft(U, axis=-1)), u[l + 1], atol=1e-12)


def test_burgers_newton_march_conserves_cell_average_mass():
    nx = 32
    u0 = dg.p2_project(lambda x: syn.fourier_u0_at(0, x), nx)
    prob = Problem(nx=nx, nt=12, t_final=0.3, alpha=0.5, beta=0.0, space="dg_p2_llf", time="bdf2")
    u = onewton.march(prob, u0)
    m = u[:, 0, :].sum(axis=-1) / nx
    np.testing.assert_allclose(m, m[0], atol=1e-13)
    assert np.all(np.isfinite(u))


def _characteristic(x, t, u0):
    """u(x, t) of Burgers before the shock: u = u0(x - u t) by fixed-point iteration."""
    u = u0(x)
    for _ in range(200):
        u = u0(x - u * t)
    return u


def test_burgers_converges_to_characteristic_solution_before_the_shock():
    """u0 = 0.5 + 0.1 sin(2 pi x) (shock at t = 1/(0.2 pi) ~ 1.6), T = 0.3, backward Euler with
    h_t = 3 h_x: cell averages converge at first order (the time error dominates)."""
    u0 = lambda x: 0.5 + 0.1 * np.sin(2 * np.pi * x)
    errs = []
    for nx in (32, 64, 128):
        nt = int(round(0.3 / (3.0 / nx)))
        prob = Problem(nx=nx, nt=nt, t_final=3.0 * nt / nx, alpha=0.5, beta=0.0, space="dg_p2_llf", time="be")
        u = onewton.march(prob, dg.p2_project(u0, nx))
        h = 1.0 / nx
        exact = dg.p2_project(lambda x: _characteristic(x, prob.t_final, u0), nx)[0]
        errs.append(np.max(np.abs(u[-1, 0] - exact)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 1.7 < r1 < 2.4 and 1.7 < r2 < 2.4, errs


@pytest.mark.parametrize("time", ["be", "bdf2"])
def test_kd_solve_matches_dense_assembly(time):
    prob = _prob(nx=8, nt=5, time=time, precond_c=0.8)
    rng = np.random.default_rng(5)
    r = rng.standard_normal((5, 3, 8))
    s = dg.p2_kd_solve(prob, r)
    K = dg.p2_kd_dense(prob)
    np.testing.assert_allclose(s.ravel(), np.linalg.solve(K, r.ravel()), rtol=1e-10, atol=1e-12)


def test_pdhg_limit_is_the_newton_march():
    nx, nt = 16, 6
    u0 = dg.p2_project(lambda x: syn.fourier_u0_at(0, x), nx)
    prob = default_constants(Problem(nx=nx, nt=nt, t_final=0.1, alpha=0.5, beta=0.0, space="dg_p2_llf",
                                     time="be"), u0)
    tu, tp, _ = opdhg.auto_steps(prob, u0)
    res = opdhg.run(prob, u0, tu, tp, eps=1e-10, max_iter=20000)
    assert res.converged
    np.testing.assert_allclose(res.u, onewton.march(prob, u0), atol=1e-9)


@pytest.mark.parametrize("nx", [16, 256, 4096])
def test_projection_of_the_seeded_fourier_sum_matches_its_closed_form(nx):
    """The quadrature projection against the exact Legendre coefficients of each sine mode
    (spherical Bessel functions), which the benchmark uses as its DG initial data."""
    a = dg.p2_project(lambda x: syn.fourier_u0_at(3, x), nx)
    b = syn.fourier_u0_legendre(3, nx)
    assert np.max(np.abs(a - b)) < 1e-13
