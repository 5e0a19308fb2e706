"""GPU parity for long time axes: 512 < N_t <= 1024 (one wavefront per spectrum
column), 1024 < N_t <= 4096 (and N_x = 8 up to 8192), where one column spans
several wavefronts of the column solve (2, 4 or 8 waves, 16 levels per lane,
wave totals exchanged through LDS), and 4096 < N_t <= 8192 with N_x >= 16, the
chunked column solve (chunks of 256 levels of 16 columns solved from zero
entering states, the states carried between chunks through the chunk maps,
every chunk solved again; for a float spectrum the low modes in FP64).  The HIP path through the C ABI against
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
    (16, 8192, "be", 1.0, 0.0), (8, 8192, "bdf2", 0.95, 0.0), (64, 4097, "bdf2", 1.0, 0.0),
    (32, 4500, "bdf2", 0.9, 1e-3), (16, 6001, "be", 0.7, 0.0), (32, 4352, "bdf2", 1.0, 0.0),
    (256, 2048, "bdf2", 1.0, 0.0), (512, 3000, "be", 0.7, 0.0), (128, 4096, "bdf2", 0.9, 1e-3)])
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
    dict(nx=64, nt=5000, t_final=2.0, alpha=0.5, beta=0.0, gamma=0.0, time="bdf2", space="fd_lf", tau=0.65, n=4),
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


def test_chunked_fp32_trajectory(gpu_lib):
    """FP32 through the chunked column solve with both of its grids: the column blocks of the
    slowly decaying low modes in FP64 and the others in float (64 x 4500, h_t = 1.3e-3: the first
    two of four blocks in FP64), against the FP64 oracle within twice the error of the CPU
    emulation that rounds where the GPU path rounds."""
    from fp32_emulation import fp32_bar, gpu_chunked_columns, gpu_fp64_modes
    cfg = dict(nx=64, nt=4500, t_final=6.0, alpha=0.5, beta=0.0, gamma=0.0, time="bdf2", space="fd_lf")
    u0 = syn.fourier_u0(7, cfg["nx"])
    oprob = default_constants(OProblem(**cfg), u0)
    assert gpu_chunked_columns(cfg["nt"], cfg["nx"]) and 0 < gpu_fp64_modes(oprob) < cfg["nx"] // 2
    n, tau = 4, 0.6
    ref = opdhg.run(oprob, u0, tau, tau, eps=0.0, max_iter=n)
    gprob = gpu_lib.Problem(dtype=torch.float32, lf_speed=oprob.lf_speed, precond_c=oprob.precond_c, **cfg)
    res = gpu_lib.Solver(gprob).solve(_dev(u0, torch.float32), tau_u=tau, tau_phi=tau, eps=0.0, max_iter=n,
                                      check_every=2)
    assert res.stats["iters"] == n
    bar_u, bar_phi = fp32_bar(oprob, u0, tau, n, ref.u, ref.phi)
    _say(f"chunked FP32 {cfg['nx']}x{cfg['nt']}: FP64 modes {gpu_fp64_modes(oprob)}, bars {bar_u:.2e} {bar_phi:.2e}")
    assert _err(res.u, ref.u, "u") < bar_u
    assert _err(res.phi, ref.phi, "phi") < bar_phi


def test_nt_above_limit_is_unsupported(gpu_lib):
    with pytest.raises(Exception, match="unsupported"):
        gpu_lib.Solver(gpu_lib.Problem(nx=16, nt=8193, t_final=1.0, dtype=torch.float64))
