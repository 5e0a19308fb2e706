"""Pins of the one-time-step solver (Algorithm 3) on the DG P1 nodal upwind scheme (oracle/onestep.py)."""
import numpy as np
import pytest

from oracle import dg1
from oracle import onestep as oos
from oracle import pdhg as opdhg
from oracle.problem import Problem, default_constants


def _u0(nx):
    x = dg1.node_x(nx)
    return 0.5 + 0.2 * np.sin(2.0 * np.pi * x) + 0.05 * np.cos(6.0 * np.pi * x)


def _prob(**kw):
    base = dict(nx=32, nt=6, t_final=0.2, alpha=0.5, beta=0.0, time="bdf2", space="dg_p1_upwind")
    base.update(kw)
    return base


@pytest.mark.parametrize("time", ["be", "bdf2"])
def test_march_ends_at_the_newton_march(time):
    u0 = _u0(32)
    p = default_constants(Problem(**_prob(time=time)), u0)
    res = oos.run(p, u0, eps=1e-12, max_iter=5000)
    assert res.converged
    assert np.max(np.abs(res.u - dg1.p1_newton_march(p, u0))) < 1e-11


def test_first_be_step_is_algorithm_1_on_one_level():
    u0 = _u0(32)
    q = default_constants(Problem(**_prob(nt=1, time="be", t_final=0.02)), u0)
    a = oos.run(q, u0, eps=0.0, max_iter=30, tau_u=0.5, tau_phi=0.5)
    b = opdhg.run(q, u0, 0.5, 0.5, eps=0.0, max_iter=30)
    assert np.max(np.abs(a.u - b.u)) < 1e-13
    assert np.max(np.abs(a.phi - b.phi)) < 1e-13


@pytest.mark.parametrize("c0", [1.0, 1.5])
def test_mode_blocks_are_the_one_level_gram(c0):
    """The per-mode 2x2 blocks, mapped back to the nodal planes by the FFT, equal the dense K_d of
    the backward-Euler problem with one level and time step h_t / c0."""
    p = Problem(**_prob(nx=8, nt=4, precond_c=0.7))
    q = p.with_(nt=1, time="be", t_final=p.ht / c0)
    kd = dg1.p1_kd_dense(q)
    rng = np.random.default_rng(3)
    r = rng.standard_normal((2, 8))
    kl = oos.dg1_step_precond(p, c0)
    R = np.fft.fft(r, axis=-1)
    S = np.fft.ifft(np.linalg.solve(kl, R.T[:, :, None])[:, :, 0].T, axis=-1).real
    np.testing.assert_allclose(S.ravel(), np.linalg.solve(kd, r.ravel()), rtol=1e-12, atol=1e-14)


def test_linear_transport_steps_keep_cell_averages():
    """f(u) = 2u: every converged step conserves the cell-average mass exactly (the upwind DG P1
    scheme is conservative), to the step tolerance."""
    u0 = _u0(32)
    p = default_constants(Problem(**_prob(alpha=0.0, beta=2.0, time="be")), u0)
    res = oos.run(p, u0, eps=1e-13, max_iter=20000)
    m = res.u.sum(axis=(1, 2))
    assert np.max(np.abs(m - m[0])) < 1e-9
