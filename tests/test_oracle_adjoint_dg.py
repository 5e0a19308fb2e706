"""Oracle pins for the implicit adjoint of the DG schemes (Sections 3.1-3.2; test infrastructure only).

dl/du0 by J(u)^T mu = dl/du (oracle/adjoint.py with the exact DG Jacobian) is checked against
  * central differences (h = 1e-6) of the oracle's Newton march, which shares no code with the
    adjoint solve, for the P2 Legendre LLF scheme and the paper's P1 nodal upwind scheme, backward
    Euler and BDF2, Burgers' flux;
  * the transpose of the linear scheme's solution map built column by column (brute force: one
    Newton march per unit initial coefficient), for linear transport, where the gradient of
    w . u^{N_t} is exactly G^T w.
"""
import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import dg, dg1
from oracle.problem import Problem


def _setup(space, time, alpha, beta, nx=16, nt=5):
    cfl = 3 if space == "dg_p2_llf" else 2
    prob = Problem(nx=nx, nt=nt, t_final=nt * cfl / nx, alpha=alpha, beta=beta, time=time, space=space)
    fn = lambda x: 0.5 + 0.2 * np.sin(2 * np.pi * x) + 0.1 * np.cos(6 * np.pi * x)
    if space == "dg_p2_llf":
        return prob, dg.p2_project(fn, nx), dg.p2_newton_march
    return prob, dg1.interpolate(fn, nx), dg1.p1_newton_march


@pytest.mark.parametrize("space", ["dg_p2_llf", "dg_p1_upwind"])
@pytest.mark.parametrize("time", ["be", "bdf2"])
def test_dg_adjoint_gradient_matches_central_differences(space, time):
    prob, u0, march = _setup(space, time, alpha=0.5, beta=0.0 if space == "dg_p2_llf" else 0.2)
    u = march(prob, u0)
    rng = np.random.default_rng(11)
    w = rng.standard_normal(u0.shape)
    g = np.zeros_like(u)
    g[-1] = w
    grad = oadj.gradient_u0(prob, u, g)
    assert grad.shape == u0.shape
    h = 1e-6
    for _ in range(6):
        v = rng.standard_normal(u0.shape)
        v /= np.linalg.norm(v)
        fdv = (np.sum(w * march(prob, u0 + h * v)[-1]) - np.sum(w * march(prob, u0 - h * v)[-1])) / (2 * h)
        assert abs(fdv - np.sum(grad * v)) <= 1e-7 * max(1.0, abs(fdv)), (fdv, np.sum(grad * v))


@pytest.mark.parametrize("space", ["dg_p2_llf", "dg_p1_upwind"])
def test_dg_adjoint_is_the_transpose_of_the_linear_solution_map(space):
    prob, u0, march = _setup(space, "bdf2", alpha=0.0, beta=1.0, nx=8, nt=4)
    n = u0.size
    G = np.empty((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        G[:, i] = march(prob, e.reshape(u0.shape))[-1].ravel()
    w = np.random.default_rng(5).standard_normal(u0.shape)
    g = np.zeros((prob.nt + 1,) + u0.shape)
    g[-1] = w
    grad = oadj.gradient_u0(prob, march(prob, u0), g)
    assert np.max(np.abs(grad.ravel() - G.T @ w.ravel())) < 1e-12 * max(1.0, np.max(np.abs(G.T @ w.ravel())))
