"""Pins of the FP64 oracle's finite-difference discretisation (CPU only).

Each test checks the oracle against something other than itself: a closed
form, brute-force finite differences, an invariant of the scheme, or the
PDE it approximates.
"""
import numpy as np
import pytest

import synthetic as syn
from oracle import closed_form, fd, newton
from oracle.problem import Problem, default_constants, time_coeffs


def _problems(nx=16, nt=5):
    u0 = syn.fourier_u0(3, nx)
    out = []
    for tm in ("be", "bdf2"):
        out.append(Problem(nx=nx, nt=nt, t_final=0.5, alpha=0.0, beta=1.3, space="fd_upwind", time=tm))
        out.append(default_constants(Problem(nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.0,
                                             space="fd_lf", time=tm), u0))
        out.append(default_constants(Problem(nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.1, gamma=1e-2,
                                             space="fd_lf", time=tm), u0))
        out.append(Problem(nx=nx, nt=nt, t_final=0.1, alpha=0.0, beta=0.0, space="heat_var", time=tm,
                           precond_gamma_hat=0.6, gamma_fn=syn.heat_gamma_at))
    return out


@pytest.mark.parametrize("prob", _problems(), ids=lambda p: f"{p.space}-{p.time}-g{p.gamma}")
def test_jacobian_matches_central_differences(prob):
    """J(u) v equals (A(u + h v) - A(u - h v)) / 2h (A is at most quadratic: exact up to rounding)."""
    rng = np.random.default_rng(0)
    u = 0.5 + 0.3 * rng.standard_normal((prob.nt + 1, prob.nx))
    v = rng.standard_normal((prob.nt, prob.nx))
    h = 1e-3
    up, um = u.copy(), u.copy()
    up[1:] += h * v
    um[1:] -= h * v
    fdiff = (fd.residual(prob, up) - fd.residual(prob, um)) / (2 * h)
    jv = fd.apply_j(prob, u, v)
    assert np.max(np.abs(fdiff - jv)) <= 1e-9 * max(1.0, np.max(np.abs(jv)))


@pytest.mark.parametrize("prob", _problems(), ids=lambda p: f"{p.space}-{p.time}-g{p.gamma}")
def test_jacobian_transpose_is_exact(prob):
    """<J v, w> = <v, J^T w> with J^T applied through apply_jt."""
    rng = np.random.default_rng(1)
    u = 0.5 + 0.3 * rng.standard_normal((prob.nt + 1, prob.nx))
    v = rng.standard_normal((prob.nt, prob.nx))
    w = rng.standard_normal((prob.nt, prob.nx))
    lhs = np.sum(fd.apply_j(prob, u, v) * w)
    rhs = np.sum(v * fd.apply_jt(prob, u, w))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)


def test_dual_operator_is_backward_sweep():
    """J^T phi at unknown level m involves only phi^{m-1}, phi^m, phi^{m+1} (BDF2) -- the
    summation-by-parts structure of Section 3.1: the dual equation for phi^{m-1}
    is explicit once phi^m, phi^{m+1} are known (backward in time)."""
    prob = default_constants(Problem(nx=12, nt=6, t_final=0.5, alpha=0.5, beta=0.0, space="fd_lf",
                                     time="bdf2"), syn.fourier_u0(0, 12))
    u = np.tile(syn.fourier_u0(0, 12), (prob.nt + 1, 1))
    jt = fd.jacobian(prob, u).T.toarray()
    n = prob.nx
    for m in range(1, prob.nt + 1):
        rows = jt[(m - 1) * n:m * n]
        nz_blocks = {c // n for c in np.nonzero(np.abs(rows).sum(axis=0))[0]}
        assert nz_blocks <= {m - 1, m, m + 1} & set(range(prob.nt))


@pytest.mark.parametrize("space", ["fd_upwind", "fd_lf"])
def test_flux_difference_conserves_mass(space):
    """sum_j F(v)_j = 0 for a periodic flux difference (telescoping sum)."""
    prob = Problem(nx=37, nt=1, alpha=0.7, beta=0.2, gamma=3e-3, space=space, lf_speed=1.1)
    v = np.random.default_rng(2).standard_normal(37)
    assert abs(np.sum(fd.flux_operator(prob, v))) <= 1e-12 * np.sum(np.abs(fd.flux_operator(prob, v)))


@pytest.mark.parametrize("space,order", [("fd_upwind", 1.0), ("fd_lf", 1.0)])
def test_flux_difference_is_consistent(space, order):
    """F(v) -> d/dx f(v) - gamma v_xx at the expected order for smooth periodic v."""
    errs = []
    for nx in (128, 256, 512, 1024):
        prob = Problem(nx=nx, nt=1, alpha=0.5, beta=0.6, gamma=2e-3, space=space, lf_speed=1.2)
        x = np.arange(nx) / nx
        v = 0.4 + 0.2 * np.sin(2 * np.pi * x)
        vx = 0.4 * np.pi * np.cos(2 * np.pi * x)
        vxx = -0.8 * np.pi ** 2 * np.sin(2 * np.pi * x)
        exact = prob.fp(v) * vx - prob.gamma * vxx
        errs.append(np.max(np.abs(fd.flux_operator(prob, v) - exact)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - order) < 0.1), rates


def test_time_matrix_matches_residual_time_part():
    """B_t U + (u^0 terms) equals A(u) when the spatial operator vanishes."""
    for tm in ("be", "bdf2"):
        prob = Problem(nx=5, nt=7, t_final=0.7, alpha=0.0, beta=0.0, space="fd_upwind", time=tm)
        rng = np.random.default_rng(4)
        u = rng.standard_normal((prob.nt + 1, prob.nx))
        r = fd.residual(prob, u)
        bu = fd.time_matrix(prob) @ u[1:]
        bu[0] += time_coeffs(tm, 0)[1] * u[0] / prob.ht
        if tm == "bdf2":
            bu[1] += time_coeffs(tm, 1)[2] * u[0] / prob.ht
        assert np.allclose(r, bu, rtol=1e-13, atol=1e-12)


def test_bdf2_is_second_order_in_time():
    """BDF2 (BE start) solution of u_t + u_x = 0 with exact space differencing error
    removed: time error ratio ~4 per halving of h_t (checked via the Fourier
    closed form of the ODE per mode)."""
    # scalar ODE y' = -lambda y solved by the oracle's time coefficients
    lam = 3.0
    errs = []
    for nt in (40, 80, 160, 320):
        ht = 1.0 / nt
        y = [1.0]
        for l in range(nt):
            c0, c1, c2 = time_coeffs("bdf2", l)
            rhs = -(c1 * y[l] + (c2 * y[l - 1] if c2 else 0.0))
            y.append(rhs / (c0 + lam * ht))
        errs.append(abs(y[-1] - np.exp(-lam)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.15), rates


def test_newton_march_matches_upwind_closed_form():
    """Linear advection, BE upwind, CFL 4 (the 64 x 32 example): u^l_j = Im(g^l e^{2 pi i x_j})."""
    prob = Problem(nx=64, nt=32, t_final=2.0, alpha=0.0, beta=1.0, space="fd_upwind", time="be")
    u = newton.march(prob, syn.sine_u0(64))
    cf = closed_form.advection_sine_solution(64, 32, 4.0)
    assert np.max(np.abs(u - cf)) < 1e-13
    g = closed_form.amplification(64, 4.0, 1)
    # hand-evaluated: |1 + 4 (1 - e^{-2 pi i / 64})| = 1.0920672...
    assert abs(abs(g) - 0.9156945) < 1e-6
    assert abs(abs(g) ** 32 - 0.0597062) < 1e-6


def test_closed_form_general_data():
    """The per-mode closed form equals the Newton march for seeded Fourier data."""
    prob = Problem(nx=48, nt=12, t_final=1.0, alpha=0.0, beta=2.0, space="fd_upwind", time="be")
    u0 = syn.fourier_u0(5, 48)
    nu = 2.0 * prob.ht / prob.hx
    assert np.max(np.abs(newton.march(prob, u0) - closed_form.advection_solution(u0, 12, nu))) < 1e-13


@pytest.mark.parametrize("tm", ["be", "bdf2"])
def test_newton_march_conserves_mass(tm):
    prob = default_constants(Problem(nx=64, nt=16, t_final=0.5, alpha=0.5, beta=0.0, gamma=1e-3,
                                     space="fd_lf", time=tm), syn.fourier_u0(1, 64))
    u = newton.march(prob, syn.fourier_u0(1, 64))
    m = fd.mass(prob, u)
    assert np.max(np.abs(m - m[0])) < 1e-13
    # residual of the implicit scheme vanishes at the march
    assert fd.wnorm(prob, fd.residual(prob, u)) < 1e-11


def _characteristic_solution(u0_fn, x, t):
    """Smooth Burgers solution u = u0(x - u t) (before shocks), by fixed-point Newton."""
    u = u0_fn(x)
    for _ in range(100):
        xi = x - u * t
        h = 1e-7
        g = u - u0_fn(xi)
        dg = 1.0 + t * (u0_fn(xi + h) - u0_fn(xi - h)) / (2 * h)
        u = u - g / dg
    return u


def test_lf_burgers_converges_to_characteristics_before_shock():
    """Implicit LF Burgers approaches the exact smooth solution at first order."""
    seed = 0
    fn = lambda x: syn.fourier_u0_at(seed, np.mod(x, 1.0))
    xs = np.linspace(0, 1, 4001)
    slope = np.gradient(fn(xs), xs)
    t_shock = -1.0 / slope.min()
    T = 0.4 * t_shock
    errs = []
    for nx in (128, 256, 512):
        nt = nx // 8
        prob = default_constants(Problem(nx=nx, nt=nt, t_final=T, alpha=0.5, beta=0.0, space="fd_lf",
                                         time="be"), syn.fourier_u0(seed, nx))
        u = newton.march(prob, syn.fourier_u0(seed, nx))
        x = np.arange(nx) / nx
        errs.append(np.max(np.abs(u[-1] - _characteristic_solution(fn, x, T))))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 0.8), (errs, rates)
