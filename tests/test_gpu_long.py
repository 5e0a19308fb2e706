"""GPU parity for long time axes: 512 < N_t <= 1024 (one wavefront per spectrum
column) and 1024 < N_t <= 8192, where one column spans several wavefronts of the
column solve (2, 4 or 8 waves, 16 levels per lane, wave totals exchanged
through LDS).  The HIP path through the C ABI against
the FP64 CPU oracle: K_d^{-1} r at 1e-10 (FP64) and 1e-5 (FP32), and Algorithm 1
trajectories (fused and unfused loop bodies) at 1e-10.  N_t values include
ragged tails (not a multiple of 1024, of 64 or of 16).
"""
import numpy as np
import pytest
import torch

import synthetic as syn
from oracle import pdhg as opdhg
from oracle import precond as opre
from oracle.problem import Problem as OProblem, default_constants

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-10, torch.float32: 1e-5}


def _say(msg):
    print(msg, flush=True)


def _dev(x, dtype):
    return torch.tensor(np.asarray(x), dtype=dtype, device="cuda")


def _err(gpu, ref, name=""):
    g = gpu.detach().cpu().double().numpy()
    e = float(np.max(np.abs(g - ref)) / max(1.0, np.max(np.abs(ref))))
    _say(f"  rel err {name}: {e:.3e}")
    return e


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nx,nt,time,c,ghat", [
    (16, 600, "bdf2", 0.8, 0.0), (64, 900, "bdf2", 1.0, 0.0), (32, 1024, "be", 0.6, 0.0),
    (16, 1025, "be", 1.0, 0.0), (8, 2048, "bdf2", 0.7, 0.0), (32, 1999, "bdf2", 0.9, 1e-3),
    (16, 3000, "be", 0.5, 0.0), (64, 4096, "bdf2", 1.0, 0.0), (8, 5003, "bdf2", 0.3, 0.0),
    (16, 8192, "be", 1.0, 0.0), (8, 8192, "bdf2", 0.95, 0.0)])
def test_precond_long_columns_match_oracle(gpu_lib, dtype, nx, nt, time, c, ghat):
    _say(f"precond long nx={nx} nt={nt} {time} c={c} ghat={ghat} {dtype}")
    pk = gpu_lib
    oprob = OProblem(nx=nx, nt=nt, t_final=0.5, time=time, precond_c=c, precond_gamma_hat=ghat)
    solver = pk.Solver(pk.Problem(nx=nx, nt=nt, t_final=0.5, time=time, dtype=dtype, precond_c=c,
                                  precond_gamma_hat=ghat))
    r = np.random.default_rng(nx + nt).standard_normal((nt, nx))
    s = solver.precond(_dev(r, dtype))
    ref = opre.kd_solve(oprob, r)
    assert _err(s, ref, "K_d^-1 r") < TOL[dtype]


LONG_TRAJ = [
    dict(nx=64, nt=2048, t_final=2.0, alpha=0.5, beta=0.0, gamma=0.0, time="bdf2", space="fd_lf", tau=0.65, n=6),
    dict(nx=64, nt=3001, t_final=2.0, alpha=0.5, beta=0.0, gamma=1e-3, time="be", space="fd_lf", tau=0.65, n=6),
    dict(nx=64, nt=8192, t_final=4.0, alpha=0.0, beta=1.0, gamma=0.0, time="be", space="fd_upwind", tau=0.65, n=3),
]


@pytest.mark.parametrize("case", range(len(LONG_TRAJ)))
def test_long_trajectory_matches_oracle_fp64(gpu_lib, case):
    """Both loop bodies (1: unfused passes, 2: fused A/B/C) against one oracle run."""
    cfg = dict(LONG_TRAJ[case])
    tau = cfg.pop("tau")
    n_iter = cfg.pop("n")
    u0 = syn.fourier_u0(case, cfg["nx"])
    oprob = default_constants(OProblem(**cfg), u0)
    ref = opdhg.run(oprob, u0, tau, tau, eps=0.0, max_iter=n_iter, record=True)
    oh = np.array(ref.history)
    gprob = gpu_lib.Problem(dtype=torch.float64, lf_speed=oprob.lf_speed, precond_c=oprob.precond_c, **cfg)
    solver = gpu_lib.Solver(gprob)
    for variant in (1, 2):
        _say(f"long trajectory case {case} nx={cfg['nx']} nt={cfg['nt']} variant {variant}")
        res = solver.solve(_dev(u0, torch.float64), tau_u=tau, tau_phi=tau, eps=0.0, max_iter=n_iter,
                           check_every=2, history=True, variant=variant)
        assert res.stats["variant"] == variant
        assert res.stats["iters"] == n_iter
        assert _err(res.u, ref.u, "u") < 1e-10
        assert _err(res.phi, ref.phi, "phi") < 1e-10
        h = res.history.cpu().numpy()
        np.testing.assert_allclose(h[1:, 0], oh[:, 1], rtol=1e-9)
        np.testing.assert_allclose(h[1:, 1], oh[:, 2], rtol=1e-9, atol=1e-14)


def test_nt_above_limit_is_unsupported(gpu_lib):
    with pytest.raises(Exception, match="unsupported"):
        gpu_lib.Solver(gpu_lib.Problem(nx=16, nt=8193, t_final=1.0, dtype=torch.float64))
