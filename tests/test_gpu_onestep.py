"""One-time-step solver (Algorithm 3) on the GPU against the oracle (oracle/onestep.py)."""
import numpy as np
import pytest
import torch

import synthetic as syn
from oracle import newton as onewton
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


def _pair(pk, nx, nt, time, space, dtype=torch.float64, T=0.5, alpha=0.5, beta=0.0, gamma=0.0, seed=0):
    if space == "fd_upwind":
        u0 = np.sin(2 * np.pi * np.arange(nx) / nx)
        op = OProblem(nx=nx, nt=nt, t_final=T, alpha=0.0, beta=1.0, time=time, space=space, precond_c=1.0)
        gp = pk.Problem(nx=nx, nt=nt, t_final=T, alpha=0.0, beta=1.0, time=time, space=space, dtype=dtype,
                        precond_c=1.0)
        return u0, op, gp
    u0 = syn.fourier_u0(seed, nx)
    op = default_constants(OProblem(nx=nx, nt=nt, t_final=T, alpha=alpha, beta=beta, gamma=gamma, time=time,
                                    space=space, precond_gamma_hat=gamma), u0)
    gp = pk.Problem(nx=nx, nt=nt, t_final=T, alpha=alpha, beta=beta, gamma=gamma, time=time, space=space,
                    dtype=dtype, lf_speed=op.lf_speed, precond_c=op.precond_c, precond_gamma_hat=gamma)
    return u0, op, gp


# nx = 64 (one wave, 1 point per lane), 256 (one wave, 4), 1024 (2 waves, 8), 2048 (4 waves, 8)
CASES = [(64, 8, "be", "fd_upwind", 0.0), (256, 6, "bdf2", "fd_lf", 0.0), (1024, 5, "be", "fd_lf", 1e-3),
         (2048, 4, "bdf2", "fd_lf", 0.0)]


@pytest.mark.parametrize("nx,nt,time,space,gamma", CASES)
def test_fixed_iteration_trajectory_matches_oracle(gpu_lib, nx, nt, time, space, gamma):
    """eps = 0: every step runs exactly max_iter iterations with the same step sizes."""
    u0, op, gp = _pair(gpu_lib, nx, nt, time, space, gamma=gamma)
    K, tau = 25, 0.6
    ref = oos.run(op, u0, eps=0.0, max_iter=K, tau_u=tau, tau_phi=tau)
    res = gpu_lib.Solver(gp).solve_onestep(_dev(u0), tau_u=tau, tau_phi=tau, eps=0.0, max_iter=K)
    assert res.stats["step_iters"] == [K] * nt
    assert _err(res.u, ref.u, "u") < 1e-10
    assert _err(res.phi, ref.phi, "phi") < 1e-10
    for (grp, grd), (orp, ord_) in zip(res.stats["step_res"], ref.step_res):
        assert grp == pytest.approx(orp, rel=1e-8, abs=1e-13) and grd == pytest.approx(ord_, rel=1e-8, abs=1e-13)


@pytest.mark.parametrize("time", ["be", "bdf2"])
def test_converged_march_matches_oracle_and_newton(gpu_lib, time):
    nx, nt = 256, 32
    u0, op, gp = _pair(gpu_lib, nx, nt, time, "fd_lf")
    tau = oos.auto_steps(op, u0)[0]
    ref = oos.run(op, u0, eps=1e-10, max_iter=2000, tau_u=tau, tau_phi=tau)
    res = gpu_lib.Solver(gp).solve_onestep(_dev(u0), tau_u=tau, tau_phi=tau, eps=1e-10, max_iter=2000)
    _say(f"  steps {res.stats['step_iters'][:6]}... oracle {ref.step_iters[:6]}...")
    assert res.status == 0
    # the stopping index can move by one where a residual sits at eps within rounding
    assert all(abs(a - b) <= 1 for a, b in zip(res.stats["step_iters"], ref.step_iters))
    assert _err(res.u, ref.u, "u vs oracle") < 1e-9
    assert _err(res.u, onewton.march(op, u0), "u vs newton") < 1e-9
    assert res.stats["mass_drift"] < 1e-10


def test_auto_step_sizes_match_the_oracle_estimate(gpu_lib):
    u0, op, gp = _pair(gpu_lib, 256, 16, "bdf2", "fd_lf")
    res = gpu_lib.Solver(gp).solve_onestep(_dev(u0), eps=1e-8, max_iter=500)
    _, _, nm = oos.auto_steps(op, u0)
    _say(f"  nu_max gpu {res.stats['nu_max']:.8f} oracle {nm:.8f}")
    # both are 200 power iterations from different start vectors; the top of the spectrum is clustered,
    # so the two estimates (each from below) agree to a fraction of a percent, not to rounding
    assert res.stats["nu_max"] == pytest.approx(nm, rel=1e-2)
    assert res.status == 0


def test_one_step_converges_where_algorithm_1_diverges(gpu_lib):
    """256 x 64 BDF2 LF Burgers, seed 1 (Algorithm 1 diverges on it): the one-step march reaches the
    Newton march of the scheme."""
    u0, op, gp = _pair(gpu_lib, 256, 64, "bdf2", "fd_lf", seed=1)
    res = gpu_lib.Solver(gp).solve_onestep(_dev(u0), eps=1e-9, max_iter=2000)
    _say(f"  status {res.status}, total iterations {res.stats['iters']}")
    assert res.status == 0
    assert _err(res.u, onewton.march(op, u0), "u vs newton") < 1e-8


def test_full_size_burgers_bdf2(gpu_lib):
    """2048 x 512 BDF2 LF Burgers to a step residual of 1e-8 (FP64).  Step l leaves a residual r_l with
    slice norm <= eps, so its error is J_l^{-1} r_l, at most (h_t / c0) |r_l| since the implicit LF step is a
    max-norm contraction; summed over the steps that is T eps in the slice norm, and the max norm of a
    grid function exceeds its slice norm by at most sqrt(N_x): bound T eps sqrt(N_x)."""
    u0, op, gp = _pair(gpu_lib, 2048, 512, "bdf2", "fd_lf")
    res = gpu_lib.Solver(gp).solve_onestep(_dev(u0), eps=1e-8, max_iter=2000)
    its = res.stats["step_iters"]
    _say(f"  status {res.status}, total {res.stats['iters']}, per step {min(its)}..{max(its)}, "
         f"{res.stats['seconds']:.3f} s")
    assert res.status == 0 and 40 <= min(its) and max(its) <= 70
    assert _err(res.u, onewton.march(op, u0), "u vs newton") < 0.5 * 1e-8 * np.sqrt(2048)


def test_fp32_trajectory(gpu_lib):
    """FP32 against the FP64 oracle, 25 iterations per step.  Each step's iterate carries the FP32
    rounding of the state (|v| eps32) amplified by the step's condition (J_l ~ (c0/h_t)(I + h_t dF)),
    a few eps32 per step, accumulated over the steps: bound 4 nt eps32 + 1e-5."""
    nx, nt = 1024, 8
    u0, op, gp = _pair(gpu_lib, nx, nt, "bdf2", "fd_lf", dtype=torch.float32)
    ref = oos.run(op, u0, eps=0.0, max_iter=25, tau_u=0.6, tau_phi=0.6)
    res = gpu_lib.Solver(gp).solve_onestep(_dev(u0, torch.float32), tau_u=0.6, tau_phi=0.6, eps=0.0, max_iter=25)
    assert _err(res.u, ref.u, "u fp32") < 4 * nt * 6e-8 + 1e-5


def test_max_iter_and_forced_divergence(gpu_lib):
    u0, op, gp = _pair(gpu_lib, 128, 6, "be", "fd_lf")
    s = gpu_lib.Solver(gp)
    r1 = s.solve_onestep(_dev(u0), tau_u=0.6, tau_phi=0.6, eps=1e-14, max_iter=3)
    assert r1.status == 1 and r1.stats["step_iters"] == [3] * 6
    # a divergence factor below 1 flags the second iteration of step 0: the march stops there
    u = torch.full((7, 128), 7.0, dtype=torch.float64, device="cuda")
    r2 = s.solve_onestep(_dev(u0), tau_u=0.6, tau_phi=0.6, eps=0.0, max_iter=50, u=u, diverge_factor=1e-3)
    assert r2.status == 2
    assert r2.stats["step_iters"] == [2, 0, 0, 0, 0, 0]
    assert torch.all(u[2:] == 7.0)
    # the handle recovers: a normal march afterwards
    r3 = s.solve_onestep(_dev(u0), tau_u=0.6, tau_phi=0.6, eps=1e-9, max_iter=1000)
    assert r3.status == 0


def test_unsupported_cases(gpu_lib):
    gp = gpu_lib.Problem(nx=32, nt=4, t_final=0.5, alpha=0.5, beta=0.0, time="be", space="fd_lf")
    with pytest.raises(gpu_lib.PdhgError):
        gpu_lib.Solver(gp).solve_onestep(_dev(syn.fourier_u0(0, 32)))
    gd = gpu_lib.Problem(nx=64, nt=4, t_final=0.5, alpha=0.5, beta=0.0, time="be", space="dg_p2_llf")
    with pytest.raises(gpu_lib.PdhgError):
        gpu_lib.Solver(gd).solve_onestep(_dev(np.zeros((3, 64))))


# ------------------------------------------------------------------ batched one-step solver
MIXED = [
    dict(nx=256, nt=9, t_final=0.1, alpha=0.5, beta=0.0, gamma=0.0, time="bdf2", space="fd_lf", seed=0),
    dict(nx=512, nt=5, t_final=0.05, alpha=0.5, beta=0.0, gamma=1e-3, precond_gamma_hat=1e-3, time="be",
         space="fd_lf", seed=2),
    dict(nx=1024, nt=6, t_final=0.2, alpha=0.0, beta=1.0, gamma=0.0, time="be", space="fd_upwind", seed=3),
    dict(nx=2048, nt=4, t_final=0.02, alpha=0.5, beta=0.0, gamma=0.0, time="bdf2", space="fd_lf", seed=4),
    dict(nx=4096, nt=3, t_final=0.01, alpha=0.5, beta=0.0, gamma=5e-4, precond_gamma_hat=5e-4, time="bdf2",
         space="fd_lf", seed=6),
]


def _batch(pk, cfgs, dtype):
    probs, u0s = [], []
    for c in cfgs:
        c = dict(c)
        seed = c.pop("seed")
        probs.append(pk.Problem(dtype=dtype, **c))
        u0s.append(syn.fourier_u0(seed, c["nx"]))
    return probs, u0s


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batch_matches_single_solves_bitwise(gpu_lib, dtype):
    """Every problem of a batch (block size set by the widest problem, idle threads past each problem's
    width) reproduces its single solve bit for bit, with given and with automatic step sizes."""
    probs, u0s = _batch(gpu_lib, MIXED, dtype)
    bs = gpu_lib.BatchSolver(probs)
    taus = [0.6, 0.5, 0.7, 0.55, 0.6]
    for tau in (taus, None):
        res = bs.solve_onestep(bs.pack_u0(u0s), tau_u=tau, tau_phi=tau, eps=1e-9 if dtype == torch.float64 else 0.0,
                               max_iter=400 if dtype == torch.float64 else 30, want_steps=True)
        for i, (p, u0) in enumerate(zip(probs, u0s)):
            st = res.stats[i]
            ref = gpu_lib.Solver(p).solve_onestep(_dev(u0, dtype), tau_u=st["tau_u"], tau_phi=st["tau_phi"],
                                                  eps=1e-9 if dtype == torch.float64 else 0.0,
                                                  max_iter=400 if dtype == torch.float64 else 30)
            if tau is None:
                assert st["nu_max"] > 0 and st["tau_u"] == pytest.approx(np.sqrt(0.95 / st["nu_max"]))
            assert st["step_iters"] == ref.stats["step_iters"]
            assert st["status"] == ref.status == (0 if dtype == torch.float64 else 1)
            assert torch.equal(res.views_u[i], ref.u) and torch.equal(res.views_phi[i], ref.phi)
    _say(f"  {len(probs)} problems bitwise equal to their single solves")


def test_batch_against_oracle(gpu_lib):
    probs, u0s = _batch(gpu_lib, MIXED[:3], torch.float64)
    bs = gpu_lib.BatchSolver(probs)
    res = bs.solve_onestep(bs.pack_u0(u0s), tau_u=[0.6] * 3, tau_phi=[0.6] * 3, eps=0.0, max_iter=20)
    for i, (c, u0) in enumerate(zip(MIXED[:3], u0s)):
        c = dict(c)
        c.pop("seed")
        op = default_constants(OProblem(**c), u0)
        ref = oos.run(op, u0, eps=0.0, max_iter=20, tau_u=0.6, tau_phi=0.6)
        assert _err(res.views_u[i], ref.u, f"batch problem {i} u") < 1e-10
        assert _err(res.views_phi[i], ref.phi, f"batch problem {i} phi") < 1e-10


def test_batch_workload_family_converges(gpu_lib):
    """Eight problems of the 256-problem Burgers family (BDF2, LF, T = 0.5; Algorithm 1 diverges on most of
    this family) in FP64: the batched one-step march converges on every one to its Newton march."""
    shapes = syn.batch_shapes(0, 256)
    pick = [0, 1, 2, 3, 43, 86, 129, 172]
    cfg = [shapes[i] for i in pick]
    probs = [gpu_lib.Problem(nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.0, time="bdf2", space="fd_lf",
                             dtype=torch.float64) for nx, nt, _ in cfg]
    u0s = [syn.fourier_u0(s, nx) for nx, _, s in cfg]
    bs = gpu_lib.BatchSolver(probs)
    res = bs.solve_onestep(bs.pack_u0(u0s), eps=1e-9, max_iter=2000)
    _say(f"  status {res.status}; iterations {[s['iters'] for s in res.stats]}; {res.stats[0]['seconds']:.3f} s")
    assert res.status == 0
    for i, ((nx, nt, _), u0) in enumerate(zip(cfg, u0s)):
        op = default_constants(OProblem(nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.0, time="bdf2",
                                        space="fd_lf"), u0)
        # slice residual <= eps per step: error <= T eps sqrt(N_x) (see the full-size test)
        assert _err(res.views_u[i], onewton.march(op, u0), f"{nx}x{nt} vs newton") < 0.5 * 1e-9 * np.sqrt(nx)
