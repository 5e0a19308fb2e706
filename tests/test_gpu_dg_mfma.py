"""The DG P2 residual with its per-cell products on the matrix cores (loop-body variant 6; FP32,
v_mfma_f32_16x16x4f32) against the FP64 oracle and against the VALU loop body (variant 4): Algorithm 1
trajectories element by element at the FP32 bar (1e-5, or twice the error of the FP32 emulation of the
oracle's iteration, tests/fp32_emulation.py), and the cases it does not cover."""
import numpy as np
import pytest
import torch

import synthetic as syn
from fp32_emulation import fp32_bar
from oracle import dg as odg
from oracle import pdhg as opdhg
from oracle.problem import Problem as OProblem, default_constants

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _err(gpu, ref, name=""):
    g = gpu.detach().cpu().double().numpy()
    e = float(np.max(np.abs(g - ref)) / max(1.0, np.max(np.abs(ref))))
    _say(f"  rel err {name}: {e:.3e}")
    return e


def _case(pk, nx, nt, time, dtype=torch.float32):
    u0 = odg.p2_project(lambda x: syn.fourier_u0_at(1, x), nx)
    cfg = dict(nx=nx, nt=nt, t_final=3.0 * nt / nx, alpha=0.5, beta=0.0, space="dg_p2_llf", time=time)
    op = default_constants(OProblem(**cfg), u0)
    return u0, op, pk.Problem(dtype=dtype, precond_c=op.precond_c, **cfg)


@pytest.mark.parametrize("nx,nt,time", [(64, 5, "be"), (64, 12, "bdf2"), (256, 9, "be"), (1024, 6, "bdf2")])
def test_mfma_residual_trajectory(gpu_lib, nx, nt, time):
    _say(f"MFMA DG residual nx={nx} nt={nt} {time}")
    u0, op, gp = _case(gpu_lib, nx, nt, time)
    tau, n = 0.4, 20
    ref = opdhg.run(op, u0, tau, tau, eps=0.0, max_iter=n)
    s = gpu_lib.Solver(gp)
    x0 = torch.tensor(u0, dtype=torch.float32, device="cuda")
    res = s.solve(x0, tau_u=tau, tau_phi=tau, eps=0.0, max_iter=n, check_every=4, variant=6)
    _say(f"  status {res.status}, {res.stats['iters']} iterations, Rp {res.stats['res_primal']:.3e}")
    assert res.stats["variant"] == 6 and res.stats["iters"] == n and res.status == 1
    bar_u, bar_phi = fp32_bar(op, u0, tau, n, ref.u, ref.phi)
    _say(f"  bars u {bar_u:.2e}, phi {bar_phi:.2e}")
    assert _err(res.u, ref.u, "u vs oracle") < bar_u
    phi_scale = float(np.max(np.abs(ref.phi)))
    e_phi = float(np.max(np.abs(res.phi.cpu().double().numpy() - ref.phi))) / phi_scale
    _say(f"  rel err phi (own scale) {e_phi:.3e}")
    assert e_phi < max(4 * bar_phi, 1e-5)
    valu = s.solve(x0, tau_u=tau, tau_phi=tau, eps=0.0, max_iter=n, check_every=4, variant=4)
    assert _err(res.u, valu.u.double().cpu().numpy(), "u vs VALU body") < bar_u


def test_mfma_variant_limits(gpu_lib):
    """FP64, DG P1, finite-difference problems and fewer than 64 cells do not take variant 6."""
    for dtype, space, nx in ((torch.float64, "dg_p2_llf", 64), (torch.float32, "dg_p1_upwind", 64),
                             (torch.float32, "fd_lf", 64), (torch.float32, "dg_p2_llf", 32)):
        p = gpu_lib.Problem(nx=nx, nt=4, t_final=0.1, alpha=0.5, beta=0.0, space=space, time="be", dtype=dtype)
        s = gpu_lib.Solver(p)
        lv = p.level_shape
        x0 = torch.full(lv, 0.5, dtype=dtype, device="cuda")
        with pytest.raises(Exception):
            s.solve(x0, tau_u=0.5, tau_phi=0.5, eps=0.0, max_iter=2, variant=6)
