"""Pins of the one-time-step oracle (Algorithm 3): it ends at the implicit scheme's solution (Newton
march; closed form for linear advection); its first backward-Euler step is Algorithm 1 on the N_t = 1
problem iterate for iterate; a linear step contracts at the rate of Proposition 2.1."""
import numpy as np
import pytest

import synthetic as syn
from oracle import closed_form as ocf
from oracle import newton as onewton
from oracle import onestep as oos
from oracle import pdhg as opdhg
from oracle.problem import Problem, default_constants


def _burgers(nx, nt, time, T=0.5, gamma=0.0, seed=0):
    u0 = syn.fourier_u0(seed, nx)
    p = Problem(nx=nx, nt=nt, t_final=T, alpha=0.5, beta=0.0, gamma=gamma, time=time, space="fd_lf")
    return default_constants(p, u0), u0


@pytest.mark.parametrize("time,gamma", [("be", 0.0), ("bdf2", 0.0), ("be", 1e-3)])
def test_march_ends_at_the_newton_march(time, gamma):
    prob, u0 = _burgers(64, 16, time, gamma=gamma)
    res = oos.run(prob, u0, eps=1e-11, max_iter=5000)
    assert res.converged and not res.diverged
    # step residual <= eps in the slice norm; the implicit step is a contraction (BE with a monotone
    # flux), so the error stays at a small multiple of h_t eps per step
    np.testing.assert_allclose(res.u, onewton.march(prob, u0), atol=1e-10)
    assert all(n < 200 for n in res.step_iters)


def test_linear_advection_closed_form():
    nx, nt, T = 64, 32, 2.0
    prob = Problem(nx=nx, nt=nt, t_final=T, alpha=0.0, beta=1.0, time="be", space="fd_upwind", precond_c=1.0)
    u0 = np.sin(2 * np.pi * np.arange(nx) / nx)
    res = oos.run(prob, u0, eps=1e-12, max_iter=5000)
    assert res.converged
    ref = ocf.advection_sine_solution(nx, nt, 1.0 * prob.ht / prob.hx)
    np.testing.assert_allclose(res.u, ref, atol=1e-11)


def test_first_be_step_is_algorithm_1_on_one_level():
    prob, u0 = _burgers(32, 8, "be", T=0.25, seed=1)
    tau = 0.6
    v, phi, n, _, _ = oos.solve_step(prob, 0, u0, None, tau, tau, eps=0.0, max_iter=40)
    q = prob.with_(nt=1, t_final=prob.ht)
    ref = opdhg.run(q, u0, tau, tau, eps=0.0, max_iter=40)
    assert n == 40
    np.testing.assert_allclose(v, ref.u[1], rtol=0, atol=1e-13)
    np.testing.assert_allclose(phi, ref.phi[0], rtol=0, atol=1e-13)


def test_bdf2_step_matches_the_be_step_of_length_ht_over_c0():
    """Row l >= 1 of BDF2 is (1.5 v - 2 u^l + 0.5 u^{l-1})/h_t + F(v): the BE step of length h_t/1.5
    from the state (4 u^l - u^{l-1})/3, so the two iterations coincide from the same initial guess."""
    prob, u0 = _burgers(32, 8, "bdf2", T=0.25, seed=2)
    rng = np.random.default_rng(3)
    ul, ulm = u0 + 0.01 * rng.standard_normal(32), u0
    v, phi, _, rp, rd = oos.solve_step(prob, 1, ul, ulm, 0.5, 0.5, eps=0.0, max_iter=30)
    q = prob.with_(time="be", t_final=prob.t_final / 1.5)
    w, psi, _, rp2, rd2 = oos.solve_step(q, 0, (4 * ul - ulm) / 3.0, None, 0.5, 0.5, eps=0.0, max_iter=30,
                                         v_init=ul)
    np.testing.assert_allclose(v, w, atol=1e-13)
    np.testing.assert_allclose(phi, psi, atol=1e-13)
    assert (rp, rd) == pytest.approx((rp2, rd2), rel=1e-12)


def test_linear_step_contracts_at_the_proposition_2_1_rate():
    """For a linear step the slowest error component contracts by sqrt(1 - sigma tau nu_min) per iteration
    (Proposition 2.1).  For BE upwind J and K are circulant, so nu per Fourier mode k is
    |1/h_t + a (1 - e^{-i theta_k})/h_x|^2 / (1/h_t^2 + c^2 mu_k).  Fourier modes do not mix, and the
    mean mode is never excited (the residual and every update have zero mean), so the smallest nu over
    k != 0, at k = 1, is the one that sin(2 pi x) excites."""
    nx, nt = 64, 4
    prob = Problem(nx=nx, nt=nt, t_final=4.0 * nt / nx, alpha=0.0, beta=1.0, time="be", space="fd_upwind",
                   precond_c=1.0)
    u0 = np.sin(2 * np.pi * np.arange(nx) / nx)
    th = 2 * np.pi * np.arange(1, nx) / nx
    jk = 1 / prob.ht + (1 - np.exp(-1j * th)) / prob.hx
    nu = np.abs(jk) ** 2 / ((1 / prob.ht) ** 2 + 4 * np.sin(th / 2) ** 2 / prob.hx ** 2)
    st = 0.5
    assert st * nu.max() < 1.0
    assert np.argmin(nu) in (0, nx - 2)         # k = 1 or k = nx - 1
    rate = np.sqrt(1 - st * nu.min())
    hist = []
    oos.solve_step(prob, 0, u0, None, np.sqrt(st), np.sqrt(st), eps=0.0, max_iter=200, hist=hist)
    h = np.array(hist)
    r = np.maximum(h[:, 1], h[:, 2])
    win = (r < 1e-3) & (r > 1e-11)
    slope = np.polyfit(h[win, 0], np.log(r[win]), 1)[0]
    assert abs(np.exp(slope) - rate) < 0.01, (np.exp(slope), rate)


def test_auto_steps_bound_the_step_operators():
    prob, u0 = _burgers(64, 16, "bdf2")
    t, _, nm = oos.auto_steps(prob, u0)
    assert 0.5 < nm < 2.5 and t == pytest.approx(np.sqrt(0.95 / nm))
