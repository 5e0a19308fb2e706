"""One-time-step solver (Algorithm 3) on the DG P1 nodal upwind scheme, on the GPU against the oracle
(oracle/onestep.py) and the Newton march (oracle/dg1.py)."""
import numpy as np
import pytest
import torch

import synthetic as syn
from oracle import dg1
from oracle import onestep as oos
from oracle.problem import Problem as OProblem, default_constants

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _err(gpu, ref, name=""):
    g = gpu.detach().cpu().double().numpy()
    e = float(np.max(np.abs(g - ref)) / max(1.0, np.max(np.abs(ref))))
    _say(f"  rel err {name}: {e:.3e}")
    return e


def _dev(x, dtype=torch.float64):
    return torch.tensor(np.asarray(x), dtype=dtype, device="cuda")


def _case(pk, nx, nt, time, flux="quadratic", dtype=torch.float64, T=None):
    """Quadratic: the traffic-type flux f = -u^2/2 + u with 0.1 <= u0 <= 0.45 (f' >= 0); linear: f = 2 u."""
    alpha, beta = (-0.5, 1.0) if flux == "quadratic" else (0.0, 2.0)
    u0 = dg1.interpolate(lambda x: 0.275 + 0.175 * np.sin(2 * np.pi * x), nx)
    T = 0.5 * nt / nx if T is None else T
    op = default_constants(OProblem(nx=nx, nt=nt, t_final=T, alpha=alpha, beta=beta, space="dg_p1_upwind",
                                    time=time), u0)
    gp = pk.Problem(nx=nx, nt=nt, t_final=T, alpha=alpha, beta=beta, space="dg_p1_upwind", time=time, dtype=dtype)
    return u0, op, gp


@pytest.mark.parametrize("nx,nt,time,flux", [(64, 4, "be", "quadratic"), (128, 5, "bdf2", "quadratic"),
                                             (256, 3, "bdf2", "linear"), (1024, 2, "bdf2", "quadratic"),
                                             (4096, 2, "be", "quadratic")])
def test_fixed_iteration_trajectory_matches_oracle(gpu_lib, nx, nt, time, flux):
    u0, op, gp = _case(gpu_lib, nx, nt, time, flux)
    ref = oos.run(op, u0, eps=0.0, max_iter=25, tau_u=0.6, tau_phi=0.6)
    res = gpu_lib.Solver(gp).solve_onestep(_dev(u0), tau_u=0.6, tau_phi=0.6, eps=0.0, max_iter=25)
    assert list(res.stats["step_iters"]) == [25] * nt
    assert _err(res.u, ref.u, "u") < 1e-10
    assert _err(res.phi, ref.phi, "phi") < 1e-10


@pytest.mark.parametrize("time", ["be", "bdf2"])
def test_converged_march_matches_oracle_and_newton(gpu_lib, time):
    nx, nt = 128, 6
    u0, op, gp = _case(gpu_lib, nx, nt, time)
    ref = oos.run(op, u0, eps=1e-11, max_iter=20000)
    res = gpu_lib.Solver(gp).solve_onestep(_dev(u0), eps=1e-11, max_iter=20000)
    _say(f"  steps: GPU {list(res.stats['step_iters'])}, oracle {ref.step_iters}")
    assert res.status == 0 and ref.converged
    assert list(res.stats["step_iters"]) == list(ref.step_iters)
    assert _err(res.u, ref.u, "u") < 1e-10
    assert _err(res.u, dg1.p1_newton_march(op, u0), "u - newton") < 1e-9


def test_auto_step_sizes_match_the_oracle_estimate(gpu_lib):
    u0, op, gp = _case(gpu_lib, 256, 4, "bdf2")
    tu, _, nu = oos.auto_steps(op, u0)
    res = gpu_lib.Solver(gp).solve_onestep(_dev(u0), eps=1e-9, max_iter=5000)
    _say(f"  nu_max: GPU {res.stats['nu_max']:.6f}, oracle {nu:.6f}")
    # different power-iteration start vectors: agreement to the iteration's convergence, not to rounding
    assert abs(res.stats["nu_max"] - nu) < 1e-2 * nu
    assert res.status == 0


def test_fp32_converged_march(gpu_lib):
    """FP32 to a step residual of 1e-4: the march stays within the FP32 floor of the FP64 Newton march."""
    nx, nt = 256, 4
    u0, op, gp = _case(gpu_lib, nx, nt, "be", dtype=torch.float32)
    res = gpu_lib.Solver(gp).solve_onestep(_dev(u0, torch.float32), tau_u=0.6, tau_phi=0.6, eps=1e-4, max_iter=5000)
    assert res.status == 0
    assert _err(res.u, dg1.p1_newton_march(op, u0), "u32 - newton") < 1e-4


def test_traffic_example_dg_p1(gpu_lib):
    """The traffic example (Section 4.3) on the DG P1 scheme: Algorithm 3 at tau = 0.4, c = 1, BE,
    every step to 1e-3; the GPU's per-step counts equal the oracle's."""
    nx, nt = 256, 32
    u0 = syn.traffic_u0_at(dg1.node_x(nx, 2.0))
    kw = dict(nx=nx, nt=nt, length=2.0, t_final=1.0, alpha=-1.0, beta=1.0, time="be", space="dg_p1_upwind",
              precond_c=1.0)
    ref = oos.run(OProblem(**kw), u0, eps=1e-3, max_iter=20000, tau_u=0.4, tau_phi=0.4)
    res = gpu_lib.Solver(gpu_lib.Problem(**kw)).solve_onestep(_dev(u0), tau_u=0.4, tau_phi=0.4, eps=1e-3,
                                                              max_iter=20000)
    _say(f"  DG P1 traffic one-step: GPU {res.stats['iters']}, oracle {sum(ref.step_iters)} (paper 8627)")
    assert res.status == 0 and ref.converged
    assert list(res.stats["step_iters"]) == list(ref.step_iters)
    assert _err(res.u, ref.u, "u") < 1e-10
