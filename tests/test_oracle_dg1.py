"""Pins of the DG P1 nodal upwind oracle (oracle/dg1.py): the matrices the paper prints for the
linear (A_1, A_2) and quadratic (C_1..C_9) systems, the errors of Table 2, the exact Jacobian,
conservation, the dense preconditioner, and the PDHG limit."""
import json
import os

import numpy as np
import pytest

from oracle import dg1
from oracle import newton as onewton
from oracle import pdhg as opdhg
from oracle.problem import Problem, default_constants

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _mats():
    with open(os.path.join(GOLD, "dg_p1_matrices.json")) as f:
        return {k: np.array(v) for k, v in json.load(f).items() if not k.startswith("citation")}


def test_linear_blocks_are_the_printed_A1_A2():
    m = _mats()
    for alpha, nx in ((2.0, 16), (0.7, 40)):
        p = Problem(nx=nx, nt=4, alpha=0.0, beta=alpha, space="dg_p1_upwind")
        D, L = dg1.spatial_blocks(p, np.zeros((2, nx)))
        # dv/dt = -F(v): A_1 = -dF/dv_j, A_2 = -dF/dv_{j-1}
        np.testing.assert_allclose(-D[3], m["A1"] * alpha / p.hx, rtol=1e-13)
        np.testing.assert_allclose(-L[3], m["A2"] * alpha / p.hx, rtol=1e-13)


def test_quadratic_system_is_the_printed_C_matrices():
    m = _mats()
    rng = np.random.default_rng(4)
    nx, alpha, beta = 12, -1.0, 1.0          # the traffic flux of Section 4.3
    p = Problem(nx=nx, nt=2, length=2.0, alpha=alpha, beta=beta, space="dg_p1_upwind")
    v = rng.uniform(0.0, 0.4, (2, nx))
    rhs = -dg1.spatial_operator(p, v)
    a, b, h = alpha / p.hx, beta / p.hx, p.hx
    for j in range(nx):
        um, uj = v[:, (j - 1) % nx], v[:, j]
        ref = (a * np.array([um @ m["C1"] @ um, um @ m["C2"] @ um]) + a * np.array([uj @ m["C3"] @ uj, uj @ m["C4"] @ uj])
               + b * m["C7"] @ um + b * m["C8"] @ uj)
        np.testing.assert_allclose(rhs[:, j], ref, rtol=1e-12, atol=1e-12)


def test_table2_errors():
    """Table 2: BDF2 + P1 DG for u_t + 2 u_x = 0, sin(2 pi x), T = 0.5, alpha h_t / h_x = 2."""
    with open(os.path.join(GOLD, "table2_dg_p1_errors.json")) as f:
        gold = json.load(f)
    errs = []
    for h in gold["h"]:
        nx = int(round(1.0 / h))
        p = Problem(nx=nx, nt=int(round(0.5 / h)), t_final=0.5, alpha=0.0, beta=2.0, time="bdf2",
                    space="dg_p1_upwind")
        u0 = dg1.interpolate(lambda x: np.sin(2 * np.pi * x), nx)
        u = onewton.march(p, u0)
        errs.append(dg1.space_time_error(p, u, lambda x, t: np.sin(2 * np.pi * (x - 2.0 * t))))
    assert [round(e, 4) for e in errs] == gold["error"]
    rates = [np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])]
    assert rates == pytest.approx(gold["rate_log2"], abs=0.01)


def test_jacobian_against_central_differences():
    rng = np.random.default_rng(1)
    p = Problem(nx=10, nt=3, t_final=0.3, alpha=0.5, beta=0.2, time="bdf2", space="dg_p1_upwind")
    u = 0.5 + 0.2 * rng.standard_normal((4, 2, 10))
    d = rng.standard_normal((3, 2, 10))
    jd = dg1.p1_apply_j(p, u, d)
    eps = 1e-6
    up, um = u.copy(), u.copy()
    up[1:] += eps * d
    um[1:] -= eps * d
    fd = (dg1.p1_residual(p, up) - dg1.p1_residual(p, um)) / (2 * eps)
    np.testing.assert_allclose(jd, fd, rtol=1e-7, atol=1e-6)
    # the transpose is the adjoint of J: <J d, w> = <d, J^T w>
    w = rng.standard_normal((3, 2, 10))
    assert np.sum(jd * w) == pytest.approx(np.sum(d * dg1.p1_apply_jt(p, u, w)), rel=1e-12)


def test_march_conserves_the_cell_averages():
    rng = np.random.default_rng(2)
    p = Problem(nx=32, nt=8, t_final=0.4, alpha=0.5, beta=0.3, time="bdf2", space="dg_p1_upwind")
    u0 = 0.6 + 0.1 * rng.standard_normal((2, 32))
    u = onewton.march(p, u0)
    mass = p.hx * 0.5 * (u[:, 0] + u[:, 1]).sum(axis=1)      # int u_h = h (v_1 + v_2) / 2 per cell
    np.testing.assert_allclose(mass, mass[0], atol=1e-13)


def test_kd_solve_against_dense():
    rng = np.random.default_rng(3)
    for time in ("be", "bdf2"):
        p = Problem(nx=8, nt=5, t_final=0.4, alpha=0.5, beta=0.0, time=time, space="dg_p1_upwind",
                    precond_c=0.8)
        r = rng.standard_normal((5, 2, 8))
        s = dg1.p1_kd_solve(p, r)
        ref = np.linalg.solve(dg1.p1_kd_dense(p), r.ravel()).reshape(r.shape)
        np.testing.assert_allclose(s, ref, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("beta,alpha", [(2.0, 0.0), (0.3, 0.5)])
def test_pdhg_limit_is_the_newton_march(beta, alpha):
    nx, nt = 16, 8
    p = Problem(nx=nx, nt=nt, t_final=0.25, alpha=alpha, beta=beta, time="bdf2", space="dg_p1_upwind")
    u0 = dg1.interpolate(lambda x: 0.6 + 0.2 * np.sin(2 * np.pi * x), nx)
    p = default_constants(p, u0)
    tu, tp, _ = opdhg.auto_steps(p, u0)
    res = opdhg.run(p, u0, tu, tp, eps=1e-10, max_iter=20000)
    assert res.converged
    np.testing.assert_allclose(res.u, onewton.march(p, u0), atol=1e-9)
