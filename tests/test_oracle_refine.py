"""Pins of the mesh-refinement oracle (Algorithm 2): the time interpolation is exact on data
linear in time; the refined solve ends at the fine scheme's solution (the Newton march); with a
single level it is Algorithm 1."""
import numpy as np
import pytest

import synthetic as syn
from oracle import newton as onewton
from oracle import pdhg as opdhg
from oracle import refine as oref
from oracle.problem import Problem, default_constants


def test_time_interpolation_is_exact_for_linear_in_time_data():
    rng = np.random.default_rng(0)
    a, b = rng.standard_normal(8), rng.standard_normal(8)
    nt, T = 4, 0.5
    t = np.arange(nt + 1) * T / nt
    u = a[None, :] + b[None, :] * t[:, None]
    phi = rng.standard_normal((nt, 8))
    uf, pf = oref.refine_in_time(u, phi)
    tf = np.arange(2 * nt + 1) * T / (2 * nt)
    np.testing.assert_allclose(uf, a[None, :] + b[None, :] * tf[:, None], atol=1e-15)
    for l in range(2 * nt):
        np.testing.assert_array_equal(pf[l], phi[l // 2])


def test_levels():
    assert oref.levels(16, 1) == [1, 2, 4, 8, 16]
    assert oref.levels(24, 3) == [3, 6, 12, 24]
    with pytest.raises(ValueError):
        oref.levels(24, 5)


@pytest.mark.parametrize("time", ["be", "bdf2"])
def test_refined_solve_ends_at_the_fine_newton_march(time):
    nx, nt = 64, 16
    u0 = syn.fourier_u0(0, nx)
    prob = default_constants(Problem(nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.0, time=time, space="fd_lf"), u0)
    res, per_level = oref.run(prob, u0, 1, eps=1e-10, coarse_eps=1e-6)
    assert [n for n, _ in per_level] == [1, 2, 4, 8, 16]
    assert res.converged
    np.testing.assert_allclose(res.u, onewton.march(prob, u0), atol=1e-8)


def test_single_level_is_algorithm_1():
    nx, nt = 32, 8
    u0 = syn.fourier_u0(1, nx)
    prob = default_constants(Problem(nx=nx, nt=nt, t_final=0.25, alpha=0.5, beta=0.0, time="bdf2", space="fd_lf"),
                             u0)
    res, _ = oref.run(prob, u0, nt, eps=0.0, max_iter=50, taus=lambda n: 0.6)
    ref = opdhg.run(prob, u0, 0.6, 0.6, eps=0.0, max_iter=50)
    np.testing.assert_array_equal(res.u, ref.u)
    np.testing.assert_array_equal(res.phi, ref.phi)
