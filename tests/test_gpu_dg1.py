"""DG P1 nodal upwind path (the paper's DG example) on the GPU against the FP64 oracle (oracle/dg1.py),
and Table 2 from the GPU solution."""
import json
import os

import numpy as np
import pytest
import torch

from fp32_emulation import fp32_bar
from oracle import dg1
from oracle import newton as onewton
from oracle import pdhg as opdhg
from oracle.problem import Problem as OProblem, default_constants

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-10, torch.float32: 1e-5}
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _say(msg):
    print(msg, flush=True)


def _err(gpu, ref, name=""):
    g = gpu.detach().cpu().double().numpy()
    e = float(np.max(np.abs(g - ref)) / max(1.0, np.max(np.abs(ref))))
    _say(f"  rel err {name}: {e:.3e}")
    return e


def _dev(x, dtype):
    return torch.tensor(np.asarray(x), dtype=dtype, device="cuda")


def _case(pk, nx, nt, time, dtype, flux="quadratic", c=None, T=None, length=1.0):
    """Quadratic: the traffic-type flux f = -u^2/2 + u with 0.1 <= u0 <= 0.45 (f' >= 0); linear: f = 2 u."""
    alpha, beta = (-0.5, 1.0) if flux == "quadratic" else (0.0, 2.0)
    u0 = dg1.interpolate(lambda x: 0.275 + 0.175 * np.sin(2 * np.pi * x / length), nx, length)
    T = 0.5 * nt / nx if T is None else T
    op = OProblem(nx=nx, nt=nt, length=length, t_final=T, alpha=alpha, beta=beta, space="dg_p1_upwind", time=time,
                  precond_c=0.0 if c is None else c)
    op = default_constants(op, u0)
    gp = pk.Problem(nx=nx, nt=nt, length=length, t_final=T, alpha=alpha, beta=beta, space="dg_p1_upwind",
                    time=time, dtype=dtype, precond_c=-1.0 if c is None else c)
    return u0, op, gp


CASES = [(16, 5, "be", "quadratic"), (64, 12, "bdf2", "quadratic"), (256, 7, "be", "linear"),
         (128, 70, "bdf2", "quadratic")]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nx,nt,time,flux", CASES)
def test_residual_and_dual_operator_match_oracle(gpu_lib, dtype, nx, nt, time, flux):
    u0, op, gp = _case(gpu_lib, nx, nt, time, dtype, flux)
    rng = np.random.default_rng(7)
    u = np.broadcast_to(u0, (nt + 1, 2, nx)) + 0.02 * rng.standard_normal((nt + 1, 2, nx))
    u[0] = u0
    phi = rng.standard_normal((nt, 2, nx))
    s = gpu_lib.Solver(gp)
    au, jt, res = s.residual(_dev(u, dtype), _dev(phi, dtype))
    ra = dg1.p1_residual(op, u)
    rj = dg1.p1_apply_jt(op, u, phi)
    assert _err(au, ra, "A(u)") < TOL[dtype]
    assert _err(jt, rj, "J^T phi") < TOL[dtype]
    assert res[0] == pytest.approx(dg1.p1_wnorm(op, ra), rel=1e-9 if dtype == torch.float64 else 1e-5)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nx,nt,time", [(16, 5, "be"), (64, 12, "bdf2"), (32, 200, "be")])
def test_precond_matches_oracle(gpu_lib, dtype, nx, nt, time):
    u0, op, gp = _case(gpu_lib, nx, nt, time, dtype, c=0.8)
    r = np.random.default_rng(8).standard_normal((nt, 2, nx))
    out = gpu_lib.Solver(gp).precond(_dev(r, dtype))
    assert _err(out, dg1.p1_kd_solve(op, r), "K_d^-1 r") < (1e-10 if dtype == torch.float64 else 1e-5)


@pytest.mark.parametrize("n_iter", [1, 10, 100])
@pytest.mark.parametrize("nx,nt,time,flux", [(16, 6, "be", "quadratic"), (32, 8, "bdf2", "linear"),
                                             (128, 9, "bdf2", "quadratic")])
def test_trajectory_matches_oracle_fp64(gpu_lib, nx, nt, time, flux, n_iter):
    u0, op, gp = _case(gpu_lib, nx, nt, time, torch.float64, flux)
    tau = 0.6
    ref = opdhg.run(op, u0, tau, tau, eps=0.0, max_iter=n_iter, record=True)
    res = gpu_lib.Solver(gp).solve(_dev(u0, torch.float64), tau_u=tau, tau_phi=tau, eps=0.0, max_iter=n_iter,
                                   check_every=4, history=True)
    assert res.stats["iters"] == n_iter and res.stats["variant"] == 4
    assert _err(res.u, ref.u, "u") < 1e-10
    assert _err(res.phi, ref.phi, "phi") < 1e-10
    h = res.history.cpu().numpy()
    oh = np.array(ref.history)
    np.testing.assert_allclose(h[1:, 0], oh[:, 1], rtol=1e-9)
    np.testing.assert_allclose(h[1:, 1], oh[:, 2], rtol=1e-9, atol=1e-14)


def test_converges_to_newton_march(gpu_lib):
    u0, op, gp = _case(gpu_lib, 64, 16, "bdf2", torch.float64)
    res = gpu_lib.Solver(gp).solve(_dev(u0, torch.float64), eps=1e-10, max_iter=50000, check_every=32)
    _say(f"  n* {res.stats['iters']}, tau {res.stats['tau_u']:.4f}, mass drift {res.stats['mass_drift']:.2e}")
    assert res.status == 0
    assert _err(res.u, onewton.march(op, u0), "u - newton") < 1e-8
    assert res.stats["mass_drift"] < 1e-10   # h_x sum of the cell averages (v_1 + v_2) / 2 per level


def test_table2_from_the_gpu_solution(gpu_lib):
    """Table 2: u_t + 2 u_x = 0, u0 = sin(2 pi x), T = 0.5, P1 nodal upwind DG with BDF2, h_t = h_x; the
    GPU primal-dual solution (FP64, residual 1e-11) has the printed space-time L2 errors."""
    with open(os.path.join(GOLD, "table2_dg_p1_errors.json")) as f:
        gold = json.load(f)
    errs = []
    for h in gold["h"]:
        nx, nt = int(round(1.0 / h)), int(round(0.5 / h))
        u0 = dg1.interpolate(lambda x: np.sin(2 * np.pi * x), nx)
        op = OProblem(nx=nx, nt=nt, t_final=0.5, alpha=0.0, beta=2.0, time="bdf2", space="dg_p1_upwind")
        gp = gpu_lib.Problem(nx=nx, nt=nt, t_final=0.5, alpha=0.0, beta=2.0, time="bdf2", space="dg_p1_upwind")
        res = gpu_lib.Solver(gp).solve(_dev(u0, torch.float64), eps=1e-11, max_iter=200000, check_every=64)
        assert res.status == 0
        e = dg1.space_time_error(op, res.u.cpu().numpy(), lambda x, t: np.sin(2 * np.pi * (x - 2.0 * t)))
        _say(f"  h = {h}: {nx} x {nt}, n* {res.stats['iters']}, e_h = {e:.6f}")
        errs.append(e)
    assert [round(e, 4) for e in errs] == gold["error"]


def test_trajectory_fp32(gpu_lib):
    u0, op, gp = _case(gpu_lib, 32, 8, "bdf2", torch.float32)
    tau, n = 0.6, 30
    ref = opdhg.run(op, u0, tau, tau, eps=0.0, max_iter=n)
    res = gpu_lib.Solver(gp).solve(_dev(u0, torch.float32), tau_u=tau, tau_phi=tau, eps=0.0, max_iter=n,
                                   check_every=4)
    # 1e-5, or twice the error of the FP32-storage emulation where the rounding of phibar, amplified
    # by tau times the row sum of |J^T| (4/h_t and the DG flux part), makes that larger
    bar_u, bar_phi = fp32_bar(op, u0, tau, n, ref.u, ref.phi)
    _say(f"  bars u {bar_u:.2e}, phi {bar_phi:.2e}")
    assert _err(res.u, ref.u, "u") < bar_u
    assert _err(res.phi, ref.phi, "phi") < bar_phi
