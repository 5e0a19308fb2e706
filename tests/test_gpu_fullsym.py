"""Full-symbol preconditioner K = J_c J_c^T on the GPU against the oracle (oracle/precond.py)."""
import numpy as np
import pytest
import torch

import synthetic as syn
from oracle import newton as onewton
from oracle import onestep as oos
from oracle import pdhg as opdhg
from oracle.precond import kd_full_solve
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


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nx,nt,time,space,ghat", [(64, 12, "be", "fd_lf", 0.0), (128, 37, "bdf2", "fd_lf", 0.0),
                                                   (256, 9, "bdf2", "fd_upwind", 0.0), (64, 1000, "be", "fd_lf", 0.0),
                                                   (512, 70, "bdf2", "fd_lf", 1e-3)])
def test_precond_matches_oracle(gpu_lib, dtype, nx, nt, time, space, ghat):
    kw = dict(nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.0, time=time, space=space, lf_speed=0.8, precond_c=0.6,
              precond_gamma_hat=ghat, precond_kind="full")
    op = OProblem(**kw)
    gp = gpu_lib.Problem(dtype=dtype, **kw)
    r = np.random.default_rng(3).standard_normal((nt, nx))
    out = gpu_lib.Solver(gp).precond(_dev(r, dtype))
    assert _err(out, kd_full_solve(op, r), "K_full^-1 r") < (1e-10 if dtype == torch.float64 else 1e-5)


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("nx,nt,time", [(64, 16, "bdf2"), (256, 33, "be")])
def test_trajectory_matches_oracle(gpu_lib, variant, nx, nt, time):
    u0 = syn.fourier_u0(0, nx)
    op = default_constants(OProblem(nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.0, time=time, space="fd_lf",
                                    precond_kind="full"), u0)
    gp = gpu_lib.Problem(nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.0, time=time, space="fd_lf", precond_kind="full")
    tau = 0.5
    ref = opdhg.run(op, u0, tau, tau, eps=0.0, max_iter=60)
    res = gpu_lib.Solver(gp).solve(_dev(u0), tau_u=tau, tau_phi=tau, eps=0.0, max_iter=60, check_every=4,
                                   variant=variant)
    assert res.stats["precond_c"] == pytest.approx(op.precond_c, rel=1e-12)
    assert _err(res.u, ref.u, "u") < 1e-10
    assert _err(res.phi, ref.phi, "phi") < 1e-10


def test_burgers_converges_in_fewer_iterations(gpu_lib):
    """256 x 64 BDF2 LF Burgers, seed 0, FP64 to 1e-8: the full symbol needs a fraction of the Gram iterations
    and ends at the Newton march."""
    nx, nt = 256, 64
    u0 = syn.fourier_u0(0, nx)
    its = {}
    for kind in ("gram", "full"):
        gp = gpu_lib.Problem(nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.0, time="bdf2", space="fd_lf",
                             precond_kind=kind)
        res = gpu_lib.Solver(gp).solve(_dev(u0), eps=1e-8, max_iter=50000, check_every=64)
        assert res.status == 0
        its[kind] = res.stats["iters"]
        op = default_constants(OProblem(nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.0, time="bdf2",
                                        space="fd_lf", precond_kind=kind), u0)
        assert _err(res.u, onewton.march(op, u0), f"{kind}: u - newton") < 1e-7
    _say(f"  iterations: gram {its['gram']}, full {its['full']}")
    assert its["full"] * 4 < its["gram"]


def test_one_step_full_symbol_matches_oracle(gpu_lib):
    nx, nt = 256, 8
    u0 = syn.fourier_u0(0, nx)
    op = default_constants(OProblem(nx=nx, nt=nt, t_final=0.5 * nt / 64, alpha=0.5, beta=0.0, time="bdf2",
                                    space="fd_lf", precond_kind="full"), u0)
    gp = gpu_lib.Problem(nx=nx, nt=nt, t_final=op.t_final, alpha=0.5, beta=0.0, time="bdf2", space="fd_lf",
                         precond_kind="full")
    ref = oos.run(op, u0, eps=0.0, max_iter=20, tau_u=0.6, tau_phi=0.6)
    res = gpu_lib.Solver(gp).solve_onestep(_dev(u0), tau_u=0.6, tau_phi=0.6, eps=0.0, max_iter=20)
    assert _err(res.u, ref.u, "u") < 1e-10
    conv = gpu_lib.Solver(gp).solve_onestep(_dev(u0), eps=1e-9, max_iter=2000)
    base = gpu_lib.Solver(gpu_lib.Problem(nx=nx, nt=nt, t_final=op.t_final, alpha=0.5, beta=0.0, time="bdf2",
                                          space="fd_lf")).solve_onestep(_dev(u0), eps=1e-9, max_iter=2000)
    _say(f"  one-step iterations: gram {base.stats['iters']}, full {conv.stats['iters']}")
    assert conv.status == 0 and conv.stats["iters"] < base.stats["iters"]
