"""GPU tests of the single-precision preconditioner for FP64 problems
(precond_kind "gram_f32"): u, phi, the residuals and both norms in FP64, the
spectral pass (forward FFT of the residual rows, column solve, inverse FFT) in
float.

The rounding of that pass is relative to the residual it transforms, so the
fixed point (A(u) = 0, the implicit scheme's solution) and the stopping test
are those of the FP64 method; only the trajectory carries FP32-sized
perturbations.  Checked against the FP64 oracle:
  * trajectories after 1, 10 and 100 iterations within the FP32 bar (1e-5
    relative to max(1, max |oracle|)); on rows of 1024 and 2048 points, where
    the float transforms' rounding reaches that size, within twice the error of
    a CPU emulation of the pass where that is larger;
  * the converged solution at 1e-8 against the oracle's Newton march at the
    bar of the FP64 solve, the oracle's residual norms of the returned (u, phi)
    within the tolerance, and the iteration count of the FP64 solve;
  * the unsupported combinations return an error.
"""
import numpy as np
import pytest
import torch

import synthetic as syn
from oracle import fd as ofd
from oracle import newton as onewton
from oracle import pdhg as opdhg
from oracle.problem import Problem as OProblem, default_constants

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _dev(x):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device="cuda")


def _err(gpu, ref, name=""):
    g = gpu.detach().cpu().double().numpy()
    e = float(np.max(np.abs(g - ref)) / max(1.0, np.max(np.abs(ref))))
    _say(f"  rel err {name}: {e:.3e}")
    return e


def _pair(pk, u0, kind="gram_f32", **cfg):
    oprob = default_constants(OProblem(**cfg), u0)
    gprob = pk.Problem(dtype=torch.float64, lf_speed=oprob.lf_speed, precond_c=oprob.precond_c,
                       precond_kind=kind, **cfg)
    return oprob, gprob


TRAJ = [
    dict(nx=128, nt=33, t_final=0.5, alpha=0.5, beta=0.0, gamma=0.0, time="bdf2", space="fd_lf"),
    dict(nx=256, nt=17, t_final=0.5, alpha=0.5, beta=0.0, gamma=1e-3, time="be", space="fd_lf"),
    dict(nx=64, nt=32, t_final=2.0, alpha=0.0, beta=1.0, gamma=0.0, time="be", space="fd_upwind"),
]


@pytest.mark.parametrize("case", range(len(TRAJ)))
def test_mixed_trajectory_within_fp32_bar(gpu_lib, case):
    cfg = TRAJ[case]
    u0 = syn.fourier_u0(case, cfg["nx"])
    oprob, gprob = _pair(gpu_lib, u0, **cfg)
    solver = gpu_lib.Solver(gprob)
    tau = 0.65
    for n in (1, 10, 100):
        _say(f"mixed trajectory case {case} n={n}")
        ref = opdhg.run(oprob, u0, tau, tau, eps=0.0, max_iter=n)
        res = solver.solve(_dev(u0), tau_u=tau, tau_phi=tau, eps=0.0, max_iter=n, check_every=8)
        assert res.stats["iters"] == n
        assert res.stats["variant"] == 2
        assert _err(res.u, ref.u, "u") < 1e-5
        assert _err(res.phi, ref.phi, "phi") < 1e-5


@pytest.mark.parametrize("nx,nt,t_final", [(1024, 1030, 1030 / 128), (1024, 1030, 2 * 1030 / 1024),
                                           (2048, 512, 0.5)])
def test_mixed_trajectory_wide_rows(gpu_lib, nx, nt, t_final):
    """Rows of 1024 and 2048 points (the last on the grid of the 2048 x 512 BDF2 workload): after 4 iterations the
    rounding of the float transforms reaches about 1e-5 of u, so the bar is the flat one or twice the
    error of the CPU emulation of the pass (float residual rows, transforms and spectrum, FP64
    recurrences and mode 0 of s), whichever is larger."""
    from fp32_emulation import float_spectrum_bar
    cfg = dict(nx=nx, nt=nt, t_final=t_final, alpha=0.5, beta=0.0, gamma=0.0, time="bdf2", space="fd_lf")
    u0 = syn.fourier_u0(13, nx)
    oprob, gprob = _pair(gpu_lib, u0, **cfg)
    tau, n = 0.6, 4
    ref = opdhg.run(oprob, u0, tau, tau, eps=0.0, max_iter=n)
    bar_u, bar_phi = float_spectrum_bar(oprob, u0, tau, n, ref.u, ref.phi)
    _say(f"mixed wide rows {nx}x{nt} T={t_final:.4f}: bars u {bar_u:.2e}, phi {bar_phi:.2e}")
    res = gpu_lib.Solver(gprob).solve(_dev(u0), tau_u=tau, tau_phi=tau, eps=0.0, max_iter=n, check_every=2)
    assert res.stats["iters"] == n
    assert _err(res.u, ref.u, "u") < bar_u
    assert _err(res.phi, ref.phi, "phi") < bar_phi


@pytest.mark.parametrize("time", ["be", "bdf2"])
def test_mixed_converges_like_fp64(gpu_lib, time):
    """256 x 64 Burgers, LF, auto steps, eps = 1e-8: same solution and iteration count as the FP64 solve."""
    cfg = dict(nx=256, nt=64, t_final=0.5, alpha=0.5, beta=0.0, gamma=0.0, time=time, space="fd_lf")
    u0 = syn.fourier_u0(0, cfg["nx"])
    oprob, gprob = _pair(gpu_lib, u0, **cfg)
    _, gprob64 = _pair(gpu_lib, u0, kind="gram", **cfg)
    eps = 1e-8
    res = gpu_lib.Solver(gprob).solve(_dev(u0), eps=eps, max_iter=40000, check_every=64)
    ref = gpu_lib.Solver(gprob64).solve(_dev(u0), eps=eps, max_iter=40000, check_every=64)
    _say(f"mixed {time}: {res.stats['iters']} iterations, FP64: {ref.stats['iters']}")
    assert res.status == 0 and ref.status == 0
    assert abs(res.stats["iters"] - ref.stats["iters"]) <= max(2, ref.stats["iters"] // 200)
    u = res.u.cpu().numpy()
    phi = res.phi.cpu().numpy()
    nw = onewton.march(oprob, u0)
    assert float(np.max(np.abs(u - nw))) < 2e-8
    # the oracle's norms of the returned iterate: the stopping test held in FP64
    assert ofd.wnorm(oprob, ofd.residual(oprob, u)) <= eps * 1.0001
    assert ofd.wnorm(oprob, ofd.apply_jt(oprob, u, phi)) <= eps * 1.0001
    assert res.stats["res_primal"] == pytest.approx(ofd.wnorm(oprob, ofd.residual(oprob, u)), rel=1e-6)
    m = ofd.mass(oprob, u)
    assert np.max(np.abs(m - m[0])) < 1e-10


def test_mixed_full_size_converges(gpu_lib):
    """The 2048 x 512 BDF2 Burgers workload to 1e-8: Newton march at the FP64 bar, FP64 iteration count."""
    cfg = dict(nx=2048, nt=512, t_final=0.5, alpha=0.5, beta=0.0, gamma=0.0, time="bdf2", space="fd_lf")
    u0 = syn.fourier_u0(0, cfg["nx"])
    oprob, gprob = _pair(gpu_lib, u0, **cfg)
    res = gpu_lib.Solver(gprob).solve(_dev(u0), eps=1e-8, max_iter=100000, check_every=128)
    _say(f"mixed full size: {res.stats['iters']} iterations, {res.stats['seconds']:.3f} s")
    assert res.status == 0, res.stats
    assert abs(res.stats["iters"] - 18086) <= 90
    nw = onewton.march(oprob, u0)
    assert float(np.max(np.abs(res.u.cpu().numpy() - nw))) < 1e-7


def test_mixed_unsupported_combinations(gpu_lib):
    pk = gpu_lib
    cfg = dict(nx=128, nt=16, t_final=0.5, alpha=0.5, beta=0.0, time="bdf2", space="fd_lf", precond_kind="gram_f32")
    with pytest.raises(pk.PdhgError, match="unsupported"):
        pk.Solver(pk.Problem(dtype=torch.float32, **cfg))
    with pytest.raises(pk.PdhgError, match="unsupported"):
        pk.Solver(pk.Problem(nx=64, nt=8, space="dg_p1_upwind", dtype=torch.float64, precond_kind="gram_f32"))
    s = pk.Solver(pk.Problem(dtype=torch.float64, **cfg))
    u0 = _dev(syn.fourier_u0(0, 128))
    with pytest.raises(pk.PdhgError, match="unsupported"):
        s.solve(u0, max_iter=4, variant=1)
    with pytest.raises(pk.PdhgError, match="unsupported"):
        s.solve_onestep(u0, max_iter=4)
    with pytest.raises(pk.PdhgError, match="unsupported"):
        s.solve_refined(u0, nt_start=4, max_iter=4)
    small = pk.Solver(pk.Problem(dtype=torch.float64, **dict(cfg, nx=32)))
    with pytest.raises(pk.PdhgError, match="unsupported"):
        small.solve(_dev(syn.fourier_u0(0, 32)), max_iter=4)


@pytest.mark.parametrize("nt,time", [(900, "bdf2"), (1500, "be"), (4500, "bdf2")])
def test_mixed_long_time_axis(gpu_lib, nt, time):
    """The float column solve for 512 < N_t <= 1024 (one wavefront per column), beyond (several
    wavefronts per column) and beyond 4096 (the chunked solve: chunks of 256 levels, the entering
    states carried through the chunk maps): 10 iterations within the FP32 bar of the FP64 oracle.  The recurrences
    run in FP64 on the float spectrum and mode 0 of s stays FP64 end to end: its rounding to float
    would be amplified up to N_t times by the time difference of the primal step (the CPU emulation
    in test_float_spectral_emulation.py shows both effects)."""
    cfg = dict(nx=64, nt=nt, t_final=nt / 256, alpha=0.5, beta=0.0, gamma=0.0, time=time, space="fd_lf")
    u0 = syn.fourier_u0(4, cfg["nx"])
    oprob, gprob = _pair(gpu_lib, u0, **cfg)
    ref = opdhg.run(oprob, u0, 0.6, 0.6, eps=0.0, max_iter=10)
    res = gpu_lib.Solver(gprob).solve(_dev(u0), tau_u=0.6, tau_phi=0.6, eps=0.0, max_iter=10, check_every=2)
    assert res.stats["iters"] == 10
    assert _err(res.u, ref.u, "u") < 1e-5
    assert _err(res.phi, ref.phi, "phi") < 1e-5
