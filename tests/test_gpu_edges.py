"""GPU parity at the edges of the supported sizes, against the FP64 CPU oracle:
N_t = 1 (one implicit step, a single row pair with one empty row), N_t = 2
(BDF2's first BDF2 row next to its backward-Euler start), N_t = 3 (a ragged row
pair), N_x = 8 (the smallest grid; unfused body) and N_x = 4096 (the largest;
eight points per thread in the FP64 row pass, the 96 KiB LDS ping-pong FFT in
float).  Tolerances: FP64 1e-10, FP32 1e-5 (single operator applications),
relative to max(1, max |oracle|).
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


def _dev(x, dtype=torch.float64):
    return torch.tensor(np.asarray(x), dtype=dtype, device="cuda")


def _err(gpu, ref, name=""):
    g = gpu.detach().cpu().double().numpy()
    e = float(np.max(np.abs(g - ref)) / max(1.0, np.max(np.abs(ref))))
    _say(f"  rel err {name}: {e:.3e}")
    return e


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nx,nt,time", [(8, 1, "be"), (8, 2, "bdf2"), (64, 1, "bdf2"), (64, 2, "bdf2"),
                                        (64, 3, "bdf2"), (4096, 2, "be"), (4096, 3, "bdf2")])
def test_precond_small_nt(gpu_lib, dtype, nx, nt, time):
    _say(f"precond edge nx={nx} nt={nt} {time} {dtype}")
    pk = gpu_lib
    oprob = OProblem(nx=nx, nt=nt, t_final=0.5, time=time, precond_c=0.8)
    solver = pk.Solver(pk.Problem(nx=nx, nt=nt, t_final=0.5, time=time, dtype=dtype, precond_c=0.8))
    r = np.random.default_rng(nx * 7 + nt).standard_normal((nt, nx))
    assert _err(solver.precond(_dev(r, dtype)), opre.kd_solve(oprob, r), "K_d^-1 r") < TOL[dtype]


EDGE_TRAJ = [
    dict(nx=64, nt=1, time="be", space="fd_lf", variants=(1, 2)),
    dict(nx=64, nt=1, time="bdf2", space="fd_upwind", variants=(1, 2)),
    dict(nx=64, nt=2, time="bdf2", space="fd_lf", variants=(1, 2)),
    dict(nx=128, nt=3, time="bdf2", space="fd_lf", variants=(1, 2)),
    dict(nx=8, nt=5, time="bdf2", space="fd_lf", variants=(1,)),
    dict(nx=4096, nt=6, time="bdf2", space="fd_lf", variants=(1, 2), t_final=12 / 4096),   # h_t = 2 h_x
]


@pytest.mark.parametrize("case", range(len(EDGE_TRAJ)))
def test_edge_trajectory_matches_oracle_fp64(gpu_lib, case):
    cfg = dict(EDGE_TRAJ[case])
    variants = cfg.pop("variants")
    cfg.setdefault("t_final", 0.5)
    cfg.update(alpha=0.5, beta=0.0) if cfg["space"] == "fd_lf" else cfg.update(alpha=0.0, beta=1.0)
    u0 = syn.fourier_u0(case, cfg["nx"])
    oprob = default_constants(OProblem(**cfg), u0)
    tau, n_iter = 0.6, 20
    ref = opdhg.run(oprob, u0, tau, tau, eps=0.0, max_iter=n_iter, record=True)
    oh = np.array(ref.history)
    solver = gpu_lib.Solver(gpu_lib.Problem(dtype=torch.float64, lf_speed=oprob.lf_speed,
                                            precond_c=oprob.precond_c, **cfg))
    for variant in variants:
        _say(f"edge trajectory {cfg} variant {variant}")
        res = solver.solve(_dev(u0), tau_u=tau, tau_phi=tau, eps=0.0, max_iter=n_iter, check_every=4,
                           history=True, variant=variant)
        assert res.stats["variant"] == variant and res.stats["iters"] == n_iter
        assert _err(res.u, ref.u, "u") < 1e-10
        assert _err(res.phi, ref.phi, "phi") < 1e-10
        h = res.history.cpu().numpy()
        np.testing.assert_allclose(h[1:, 0], oh[:, 1], rtol=1e-9)
        np.testing.assert_allclose(h[1:, 1], oh[:, 2], rtol=1e-9, atol=1e-14)


def test_mixed_at_largest_nx(gpu_lib):
    """The single-precision spectral pass at N_x = 4096 (float FFT with the 96 KiB ping-pong) stays
    within the FP32 bar of the FP64 oracle after 10 iterations."""
    cfg = dict(nx=4096, nt=9, t_final=18 / 4096, alpha=0.5, beta=0.0, time="bdf2", space="fd_lf")
    u0 = syn.fourier_u0(3, cfg["nx"])
    oprob = default_constants(OProblem(**cfg), u0)
    ref = opdhg.run(oprob, u0, 0.6, 0.6, eps=0.0, max_iter=10)
    s = gpu_lib.Solver(gpu_lib.Problem(dtype=torch.float64, lf_speed=oprob.lf_speed, precond_c=oprob.precond_c,
                                       precond_kind="gram_f32", **cfg))
    res = s.solve(_dev(u0), tau_u=0.6, tau_phi=0.6, eps=0.0, max_iter=10, check_every=2)
    assert _err(res.u, ref.u, "u") < 1e-5
    assert _err(res.phi, ref.phi, "phi") < 1e-5
