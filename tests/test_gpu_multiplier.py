"""The multiplier form of Algorithm 1 (u^0 free, lambda imposing u^0 = u0; Section 3.3) on the GPU against the
FP64 oracle (oracle/lagrange.py): trajectories element by element, the converged solution, the traffic
example's iteration count, and the unsupported combinations."""
import numpy as np
import pytest
import torch

import synthetic as syn
from oracle import lagrange as olag
from oracle import newton as onewton
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


def _pair(pk, u0, dtype=torch.float64, **cfg):
    op = default_constants(OProblem(**cfg), u0)
    gp = pk.Problem(dtype=dtype, lf_speed=op.lf_speed, precond_c=op.precond_c, **cfg)
    return op, gp


CASES = [
    dict(nx=64, nt=16, t_final=0.5, alpha=0.5, beta=0.0, gamma=0.0, time="bdf2", space="fd_lf"),
    dict(nx=128, nt=21, t_final=0.5, alpha=0.5, beta=0.0, gamma=1e-3, time="be", space="fd_lf"),
    dict(nx=64, nt=32, t_final=2.0, alpha=0.0, beta=1.0, gamma=0.0, time="be", space="fd_upwind"),
    dict(nx=256, nt=7, t_final=0.5, alpha=0.5, beta=0.0, gamma=0.0, time="bdf2", space="fd_lf"),
]


@pytest.mark.parametrize("n_iter", [1, 2, 10, 100])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_multiplier_trajectory_matches_oracle(gpu_lib, case, n_iter):
    cfg = CASES[case]
    u0 = syn.sine_u0(cfg["nx"]) if cfg["space"] == "fd_upwind" else syn.fourier_u0(case, cfg["nx"])
    op, gp = _pair(gpu_lib, u0, **cfg)
    tau, tau_u0, tau_lam = 0.6, 0.3, 0.99
    ref = olag.run(op, u0, tau, tau, tau_lam, eps=0.0, max_iter=n_iter, tau_u0=tau_u0)
    res = gpu_lib.Solver(gp).solve(torch.tensor(u0, device="cuda"), tau_u=tau, tau_phi=tau, eps=0.0,
                                   max_iter=n_iter, check_every=8, init_multiplier=True, tau_u0=tau_u0,
                                   tau_lam=tau_lam)
    assert res.stats["iters"] == n_iter and res.stats["variant"] == 2
    assert _err(res.u, ref.u, "u (u^0 included)") < 1e-10
    assert _err(res.phi, ref.phi, "phi") < 1e-10
    if n_iter > 1:
        assert float(np.max(np.abs(ref.u[0] - u0))) > 0.0   # u^0 does move


def test_multiplier_fp32_trajectory(gpu_lib):
    cfg = CASES[0]
    u0 = syn.fourier_u0(0, cfg["nx"])
    op, gp = _pair(gpu_lib, u0, dtype=torch.float32, **cfg)
    ref = olag.run(op, u0, 0.6, 0.6, 0.99, eps=0.0, max_iter=50)
    res = gpu_lib.Solver(gp).solve(torch.tensor(u0, dtype=torch.float32, device="cuda"), tau_u=0.6, tau_phi=0.6,
                                   eps=0.0, max_iter=50, init_multiplier=True)
    assert _err(res.u, ref.u, "u") < 1e-5
    assert _err(res.phi, ref.phi, "phi") < 1e-5


@pytest.mark.parametrize("time", ["be", "bdf2"])
def test_multiplier_converges_to_the_scheme(gpu_lib, time):
    """256 x 64 Burgers LF, auto steps, eps = 1e-8: the limit has u^0 = u0 and is the Newton march."""
    cfg = dict(nx=256, nt=64, t_final=0.5, alpha=0.5, beta=0.0, gamma=0.0, time=time, space="fd_lf")
    u0 = syn.fourier_u0(0, 256)
    op, gp = _pair(gpu_lib, u0, **cfg)
    res = gpu_lib.Solver(gp).solve(torch.tensor(u0, device="cuda"), eps=1e-8, max_iter=50000, check_every=64,
                                   init_multiplier=True)
    _say(f"  {time}: status {res.status} after {res.stats['iters']} iterations")
    assert res.status == 0
    u = res.u.cpu().numpy()
    assert float(np.max(np.abs(u - onewton.march(op, u0)))) < 2e-8
    assert float(np.max(np.abs(u[0] - u0))) < 2e-8


def test_multiplier_traffic_iteration_count(gpu_lib):
    """The traffic example (Section 4.3; FD upwind, BE, 256 x 32, tau = (0.4, 0.4, 0.99), c = 1, 1e-3): the
    oracle's count in the multiplier form (the paper prints 4573)."""
    kw = dict(nx=256, nt=32, length=2.0, t_final=1.0, alpha=-1.0, beta=1.0, time="be", precond_c=1.0,
              space="fd_upwind")
    u0 = syn.traffic_u0(256, 2.0)
    ref = olag.run(OProblem(**kw), u0, 0.4, 0.4, 0.99, eps=1e-3, max_iter=20000)
    res = gpu_lib.Solver(gpu_lib.Problem(**kw)).solve(torch.tensor(u0, device="cuda"), tau_u=0.4, tau_phi=0.4,
                                                      eps=1e-3, max_iter=20000, check_every=64,
                                                      init_multiplier=True, tau_lam=0.99)
    _say(f"  multiplier form: GPU n* {res.stats['iters']}, oracle {ref.iters} (u^0 fixed: "
         f"{opdhg.run(OProblem(**kw), u0, 0.4, 0.4, eps=1e-3, max_iter=20000).iters}; paper 4573)")
    assert ref.converged and res.status == 0 and res.stats["iters"] == ref.iters
    assert _err(res.u, ref.u, "u") < 1e-10


def test_multiplier_full_size(gpu_lib):
    """The 2048 x 512 BDF2 Burgers workload, 3 iterations, every element."""
    cfg = dict(nx=2048, nt=512, t_final=0.5, alpha=0.5, beta=0.0, gamma=0.0, time="bdf2", space="fd_lf")
    u0 = syn.fourier_u0(0, 2048)
    op, gp = _pair(gpu_lib, u0, **cfg)
    ref = olag.run(op, u0, 0.68, 0.68, 0.99, eps=0.0, max_iter=3)
    res = gpu_lib.Solver(gp).solve(torch.tensor(u0, device="cuda"), tau_u=0.68, tau_phi=0.68, eps=0.0, max_iter=3,
                                   check_every=128, init_multiplier=True)
    assert _err(res.u, ref.u, "u") < 1e-10
    assert _err(res.phi, ref.phi, "phi") < 1e-10


def test_multiplier_unsupported(gpu_lib):
    pk = gpu_lib
    u0 = torch.tensor(syn.fourier_u0(0, 64), device="cuda")
    s = pk.Solver(pk.Problem(nx=64, nt=8, t_final=0.5, alpha=0.5, beta=0.0, time="bdf2", space="fd_lf"))
    for kw in (dict(variant=1), dict(backoff=2)):
        with pytest.raises(pk.PdhgError, match="unsupported"):
            s.solve(u0, max_iter=4, init_multiplier=True, **kw)
    with pytest.raises(pk.PdhgError, match="unsupported"):
        pk.Solver(pk.Problem(nx=64, nt=8, space="dg_p1_upwind")).solve(
            torch.zeros((2, 64), dtype=torch.float64, device="cuda"), max_iter=4, init_multiplier=True)
