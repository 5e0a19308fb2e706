"""Failure handling of pdhg_solve, forced from the host on small problems (SURVEY-style fault tests):

* steps with sigma tau nu_max > 1 make Algorithm 1 diverge (Proposition 2.1 needs sigma tau nu < 1);
  the solve returns PDHG_DIVERGED with the last good checkpoint, which is the oracle's iterate M;
* with back-offs the solve restarts from that checkpoint with both steps times 0.7 and converges to
  the closed-form solution of the CFL-4 advection problem;
* the single-precision stop rule (scale-free tolerance or stall at the rounding floor) ends an FP32
  solve that can never reach an FP64 tolerance.
"""
import numpy as np
import pytest
import torch

import synthetic as syn
from oracle import newton as onewton
from oracle import pdhg as opdhg
from oracle.closed_form import advection_sine_solution
from oracle.problem import Problem as OProblem, default_constants

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _advection(pk):
    u0 = syn.sine_u0(64)
    op = default_constants(OProblem(nx=64, nt=32, t_final=2.0, alpha=0.0, beta=1.0, space="fd_upwind",
                                    time="be"), u0)
    gp = pk.Problem(nx=64, nt=32, t_final=2.0, alpha=0.0, beta=1.0, time="be", space="fd_upwind",
                    dtype=torch.float64, precond_c=op.precond_c)
    return u0, op, gp


@pytest.mark.parametrize("tau,chunk", [(2.0, 8), (1.43, 8)])
def test_divergence_returns_the_last_good_checkpoint(gpu_lib, tau, chunk):
    """tau = 2 (sigma tau nu_max ~ 7.9) diverges at once; tau = 1.43 (~4.03, just past the value 4 where
    the iteration map of the stiffest mode gets an eigenvalue below -1, growth ~1.2 per iteration)
    diverges only after a while, so that the checkpoint is a later iterate."""
    u0, op, gp = _advection(gpu_lib)
    res = gpu_lib.Solver(gp).solve(torch.tensor(u0, device="cuda"), tau_u=tau, tau_phi=tau, eps=1e-10,
                                   max_iter=50000, check_every=chunk)
    m = res.stats["iters"]
    _say(f"  tau {tau}: status {res.status}, returned iterate M = {m}, ||A(u)|| = {res.stats['res_primal']:.3e}")
    assert res.status == 2
    assert m == 0 or m % chunk == chunk - 1
    if tau < 1.0:
        assert m > 0
    ref = opdhg.run(op, u0, tau, tau, eps=0.0, max_iter=m)
    su = max(1.0, float(np.max(np.abs(ref.u))))
    assert float(np.max(np.abs(res.u.cpu().numpy() - ref.u))) < 1e-10 * su
    assert float(np.max(np.abs(res.phi.cpu().numpy() - ref.phi))) < 1e-10 * max(1.0, float(np.max(np.abs(ref.phi))))
    assert np.isfinite(res.stats["res_primal"]) and np.isfinite(res.stats["res_dual"])
    if m > 0:
        assert res.stats["res_primal"] == pytest.approx(ref.res_primal, rel=1e-9)


def test_backoff_restarts_from_the_checkpoint_and_converges(gpu_lib):
    u0, op, gp = _advection(gpu_lib)
    res = gpu_lib.Solver(gp).solve(torch.tensor(u0, device="cuda"), tau_u=2.0, tau_phi=2.0, eps=1e-10,
                                   max_iter=20000, check_every=8, backoff=5)
    tau = res.stats["tau_u"]
    k = round(np.log(tau / 2.0) / np.log(0.7))
    _say(f"  status {res.status} after {k} back-offs, tau {tau:.4f}, {res.stats['iters']} iterations")
    assert res.status == 0
    assert 1 <= k <= 5 and tau == pytest.approx(2.0 * 0.7 ** k, rel=1e-12)
    assert float(np.max(np.abs(res.u.cpu().numpy() - advection_sine_solution(64, 32, 4.0)))) < 1e-9


def test_single_precision_stop_rule(gpu_lib):
    """FP32, 256 x 64 BDF2 Burgers: eps = 1e-8 is below the FP32 rounding floor; the stop rule ends the
    solve (converged on the scale-free tolerance, or stalled), near the FP64 Newton march."""
    nx, nt = 256, 64
    u0 = syn.fourier_u0(0, nx)
    op = default_constants(OProblem(nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.0, time="bdf2",
                                    space="fd_lf"), u0)
    gp = gpu_lib.Problem(nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.0, time="bdf2", space="fd_lf",
                         dtype=torch.float32)
    s = gpu_lib.Solver(gp)
    x = torch.tensor(u0, dtype=torch.float32, device="cuda")
    plain = s.solve(x, eps=1e-8, max_iter=20000, check_every=64)
    assert plain.status == 1   # FP32 cannot reach 1e-8
    res = s.solve(x, eps=1e-8, max_iter=20000, check_every=64, eps_rel=1e-6, stall_iters=500)
    err = float(np.max(np.abs(res.u.cpu().double().numpy() - onewton.march(op, u0))))
    _say(f"  stop rule: status {res.status} after {res.stats['iters']} iterations, "
         f"||A(u)|| = {res.stats['res_primal']:.3e}, max |u - newton| = {err:.3e}")
    assert res.status in (0, 3)
    assert res.stats["iters"] < 20000
    assert err < 1e-4
