"""Mesh refinement in time (Algorithm 2) on the GPU against the oracle (oracle/refine.py)."""
import numpy as np
import pytest
import torch

import synthetic as syn
from oracle import dg as odg
from oracle import newton as onewton
from oracle import refine as oref
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


@pytest.mark.parametrize("time,nt,nt_start", [("bdf2", 16, 1), ("be", 24, 3)])
def test_refined_trajectory_matches_oracle(gpu_lib, time, nt, nt_start):
    nx = 64
    u0 = syn.fourier_u0(0, nx)
    op = default_constants(OProblem(nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.0, time=time, space="fd_lf"), u0)
    ref, per_level = oref.run(op, u0, nt_start, eps=0.0, max_iter=40, coarse_eps=0.0, coarse_max_iter=30,
                              taus=lambda n: 0.6)
    gp = gpu_lib.Problem(nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.0, time=time, space="fd_lf",
                         lf_speed=op.lf_speed, precond_c=op.precond_c)
    res = gpu_lib.Solver(gp).solve_refined(_dev(u0), nt_start=nt_start, coarse_max_iter=30, coarse_eps=0.0,
                                           tau_u=0.6, tau_phi=0.6, eps=0.0, max_iter=40, check_every=4)
    assert res.stats["level_iters"] == [n for _, n in per_level]
    assert _err(res.u, ref.u, "u") < 1e-10
    assert _err(res.phi, ref.phi, "phi") < 1e-10


def test_refinement_stabilises_a_diverging_burgers_problem(gpu_lib):
    """256 x 64, BDF2, LF, T = 0.5, seed 1: Algorithm 1 diverges; Algorithm 2 from one level converges
    to the Newton march of the fine scheme."""
    nx, nt = 256, 64
    u0 = syn.fourier_u0(1, nx)
    op = default_constants(OProblem(nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.0, time="bdf2", space="fd_lf"), u0)
    gp = gpu_lib.Problem(nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.0, time="bdf2", space="fd_lf")
    s = gpu_lib.Solver(gp)
    van = s.solve(_dev(u0), eps=1e-8, max_iter=50000, check_every=64)
    _say(f"  vanilla: status {van.status} n* {van.stats['iters']}")
    assert van.status == 2
    res = s.solve_refined(_dev(u0), nt_start=1, eps=1e-8, max_iter=50000, check_every=64)
    _say(f"  refined: status {res.status}, iterations per level {res.stats['level_iters']}")
    assert res.status == 0
    assert _err(res.u, onewton.march(op, u0), "u - newton") < 1e-6


def test_refined_dg(gpu_lib):
    nx, nt = 64, 8
    u0 = odg.p2_project(lambda x: syn.fourier_u0_at(0, x), nx)
    op = default_constants(OProblem(nx=nx, nt=nt, t_final=3.0 * nt / nx, alpha=0.5, beta=0.0, space="dg_p2_llf",
                                    time="be"), u0)
    ref, per_level = oref.run(op, u0, 2, eps=0.0, max_iter=25, coarse_eps=0.0, coarse_max_iter=20,
                              taus=lambda n: 0.6)
    gp = gpu_lib.Problem(nx=nx, nt=nt, t_final=op.t_final, alpha=0.5, beta=0.0, time="be", space="dg_p2_llf")
    res = gpu_lib.Solver(gp).solve_refined(_dev(u0), nt_start=2, coarse_max_iter=20, coarse_eps=0.0, tau_u=0.6,
                                           tau_phi=0.6, eps=0.0, max_iter=25, check_every=4)
    assert res.stats["level_iters"] == [n for _, n in per_level]
    assert _err(res.u, ref.u, "u") < 1e-10
    assert _err(res.phi, ref.phi, "phi") < 1e-10
