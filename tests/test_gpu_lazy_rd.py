"""The dual residual ||J(u)^T phi|| is evaluated only where the stopping test or
the stats need it (the previous primal residual at or below eps, or the last
iteration allowed) unless a residual history is recorded.  For every loop body
(fused and unfused finite differences, DG P2, DG P1) a solve without a history
must return bitwise the iterate, n* and norms of the same solve with one, where
the dual residual is evaluated every iteration; both are checked against the
oracle's Newton march of the scheme.
"""
import numpy as np
import pytest
import torch

import synthetic as syn
from oracle import dg as odg
from oracle import dg1
from oracle import newton as onewton
from oracle.problem import Problem as OProblem, default_constants

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _fd(pk, variant):
    nx, nt = 64, 16
    u0 = syn.fourier_u0(2, nx)
    op = default_constants(OProblem(nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.0, time="bdf2", space="fd_lf"),
                           u0)
    gp = pk.Problem(nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.0, time="bdf2", space="fd_lf",
                    dtype=torch.float64)
    return u0, op, gp, dict(variant=variant)


def _dg2(pk):
    nx, nt = 32, 8
    u0 = odg.p2_project(lambda x: syn.fourier_u0_at(0, x), nx)
    op = default_constants(OProblem(nx=nx, nt=nt, t_final=3.0 * nt / nx, alpha=0.5, beta=0.0, space="dg_p2_llf",
                                    time="be"), u0)
    gp = pk.Problem(nx=nx, nt=nt, t_final=3.0 * nt / nx, alpha=0.5, beta=0.0, space="dg_p2_llf", time="be",
                    dtype=torch.float64)
    return u0, op, gp, {}


def _dg1(pk):
    nx, nt = 32, 8
    u0 = dg1.interpolate(lambda x: 0.275 + 0.175 * np.sin(2 * np.pi * x), nx, 1.0)
    op = default_constants(OProblem(nx=nx, nt=nt, t_final=0.5 * nt / nx, alpha=-0.5, beta=1.0,
                                    space="dg_p1_upwind", time="bdf2"), u0)
    gp = pk.Problem(nx=nx, nt=nt, t_final=0.5 * nt / nx, alpha=-0.5, beta=1.0, space="dg_p1_upwind", time="bdf2",
                    dtype=torch.float64)
    return u0, op, gp, {}


@pytest.mark.parametrize("body", ["fd_unfused", "fd_fused", "dg_p2", "dg_p1"])
def test_solve_without_history_equals_solve_with_history(gpu_lib, body):
    pk = gpu_lib
    u0, op, gp, kw = {"fd_unfused": lambda: _fd(pk, 1), "fd_fused": lambda: _fd(pk, 2),
                      "dg_p2": lambda: _dg2(pk), "dg_p1": lambda: _dg1(pk)}[body]()
    s = pk.Solver(gp)
    x0 = torch.tensor(np.asarray(u0), dtype=torch.float64, device="cuda")
    a = s.solve(x0, eps=1e-9, max_iter=40000, check_every=32, **kw)
    b = s.solve(x0, eps=1e-9, max_iter=40000, check_every=32, history=True, **kw)
    _say(f"{body}: n* {a.stats['iters']} / {b.stats['iters']}, variant {a.stats['variant']}")
    assert a.status == 0 and b.status == 0
    assert a.stats["iters"] == b.stats["iters"]
    assert torch.equal(a.u, b.u) and torch.equal(a.phi, b.phi)
    assert (a.stats["res_primal"], a.stats["res_dual"]) == (b.stats["res_primal"], b.stats["res_dual"])
    nw = onewton.march(op, u0)
    assert float(np.max(np.abs(a.u.cpu().numpy() - nw))) < 1e-8
