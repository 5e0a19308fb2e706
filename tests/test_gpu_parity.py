"""GPU parity tests: the HIP path through the C ABI against the FP64 CPU oracle.

Tolerances (relative to the max-norm of the oracle result, floor 1):
FP64 1e-10, FP32 1e-5.  Sizes span several tiles and ragged tails (odd N_t,
N_t not a multiple of the column-solve segment length).
"""
import numpy as np
import pytest
import torch

import synthetic as syn
from fp32_emulation import fp32_bar
from oracle import adjoint as oadj
from oracle import fd as ofd
from oracle import newton as onewton
from oracle import pdhg as opdhg
from oracle import precond as opre
from oracle.closed_form import advection_sine_solution
from oracle.problem import Problem as OProblem, default_constants

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-10, torch.float32: 1e-5}


def _say(msg):
    print(msg, flush=True)


def _pair(pk, nx, nt, t_final, alpha, beta, gamma, time, space, dtype, u0, c=0.0, ghat=0.0, lf=0.0):
    oprob = OProblem(nx=nx, nt=nt, t_final=t_final, alpha=alpha, beta=beta, gamma=gamma, time=time,
                     space=space, lf_speed=lf, precond_c=c, precond_gamma_hat=ghat)
    oprob = default_constants(oprob, u0)
    gprob = pk.Problem(nx=nx, nt=nt, t_final=t_final, alpha=alpha, beta=beta, gamma=gamma, time=time,
                       space=space, dtype=dtype, lf_speed=oprob.lf_speed, precond_c=oprob.precond_c,
                       precond_gamma_hat=ghat)
    return oprob, gprob


def _err(gpu, ref, name=""):
    g = gpu.detach().cpu().double().numpy()
    e = float(np.max(np.abs(g - ref)) / max(1.0, np.max(np.abs(ref))))
    _say(f"  rel err {name}: {e:.3e}")
    return e


def _dev(x, dtype):
    return torch.tensor(np.asarray(x), dtype=dtype, device="cuda")


# ------------------------------------------------------------------ preconditioner
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nx,nt,time,c,ghat", [
    (8, 3, "be", 1.0, 0.0), (16, 7, "bdf2", 0.7, 0.05), (64, 32, "be", 1.0, 0.0),
    (256, 33, "bdf2", 0.9, 0.0), (512, 100, "be", 0.0, 0.6), (2048, 512, "bdf2", 0.95, 0.0),
    (4096, 64, "be", 0.5, 1e-3)])
def test_precond_matches_oracle(gpu_lib, dtype, nx, nt, time, c, ghat):
    _say(f"precond nx={nx} nt={nt} {time} c={c} ghat={ghat} {dtype}")
    pk = gpu_lib
    oprob = OProblem(nx=nx, nt=nt, t_final=0.5, time=time, precond_c=c, precond_gamma_hat=ghat)
    solver = pk.Solver(pk.Problem(nx=nx, nt=nt, t_final=0.5, time=time, dtype=dtype, precond_c=c,
                                  precond_gamma_hat=ghat))
    r = np.random.default_rng(nx + nt).standard_normal((nt, nx))
    s = solver.precond(_dev(r, dtype))
    ref = opre.kd_solve(oprob, r)
    assert _err(s, ref, "K_d^-1 r") < TOL[dtype]


# ------------------------------------------------------------------ residual and J^T
CASES = [
    dict(nx=64, nt=32, t_final=2.0, alpha=0.0, beta=1.0, gamma=0.0, time="be", space="fd_upwind"),
    dict(nx=128, nt=33, t_final=0.5, alpha=0.5, beta=0.0, gamma=0.0, time="bdf2", space="fd_lf"),
    dict(nx=256, nt=17, t_final=0.5, alpha=0.5, beta=0.0, gamma=1e-3, time="be", space="fd_lf"),
    dict(nx=32, nt=5, t_final=0.3, alpha=0.3, beta=0.4, gamma=2e-3, time="bdf2", space="fd_upwind"),
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_residual_and_dual_operator_match_oracle(gpu_lib, dtype, case):
    cfg = CASES[case]
    _say(f"residual case {cfg} {dtype}")
    u0 = syn.fourier_u0(case, cfg["nx"])
    oprob, gprob = _pair(gpu_lib, dtype=dtype, u0=u0, **cfg)
    solver = gpu_lib.Solver(gprob)
    rng = np.random.default_rng(case)
    u = 0.5 + 0.2 * rng.standard_normal((cfg["nt"] + 1, cfg["nx"]))
    phi = rng.standard_normal((cfg["nt"], cfg["nx"]))
    au, jt, res = solver.residual(_dev(u, dtype), _dev(phi, dtype))
    r_ref = ofd.residual(oprob, u)
    j_ref = ofd.apply_jt(oprob, u, phi)
    assert _err(au, r_ref, "A(u)") < TOL[dtype]
    assert _err(jt, j_ref, "J^T phi") < TOL[dtype]
    assert res[0] == pytest.approx(ofd.wnorm(oprob, r_ref), rel=TOL[dtype])
    assert res[1] == pytest.approx(ofd.wnorm(oprob, j_ref), rel=TOL[dtype])
    out = solver.apply_jt(_dev(u, dtype), _dev(phi, dtype))
    assert _err(out, j_ref, "J^T phi (adjoint apply)") < TOL[dtype]


# ------------------------------------------------------------------ trajectory
TRAJ = [
    dict(nx=64, nt=32, t_final=2.0, alpha=0.0, beta=1.0, gamma=0.0, time="be", space="fd_upwind", tau=0.7),
    dict(nx=64, nt=16, t_final=0.5, alpha=0.5, beta=0.0, gamma=0.0, time="bdf2", space="fd_lf", tau=0.65),
    dict(nx=128, nt=21, t_final=0.5, alpha=0.5, beta=0.0, gamma=1e-3, time="be", space="fd_lf", tau=0.65),
]


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("n_iter", [1, 2, 10, 100])
@pytest.mark.parametrize("case", range(len(TRAJ)))
def test_solve_trajectory_matches_oracle_fp64(gpu_lib, case, n_iter, variant):
    cfg = dict(TRAJ[case])
    tau = cfg.pop("tau")
    _say(f"trajectory case {case} n={n_iter} variant {variant}")
    u0 = syn.sine_u0(cfg["nx"]) if case == 0 else syn.fourier_u0(case, cfg["nx"])
    oprob, gprob = _pair(gpu_lib, dtype=torch.float64, u0=u0, **cfg)
    ref = opdhg.run(oprob, u0, tau, tau, eps=0.0, max_iter=n_iter, record=True)
    solver = gpu_lib.Solver(gprob)
    res = solver.solve(_dev(u0, torch.float64), tau_u=tau, tau_phi=tau, eps=0.0, max_iter=n_iter,
                       check_every=8, history=True, variant=variant)
    assert res.stats["variant"] == variant
    assert res.stats["iters"] == n_iter
    assert res.status == 1   # max_iter reached
    assert _err(res.u, ref.u, "u") < 1e-10
    assert _err(res.phi, ref.phi, "phi") < 1e-10
    h = res.history.cpu().numpy()
    oh = np.array(ref.history)
    np.testing.assert_allclose(h[1:, 0], oh[:, 1], rtol=1e-9)
    np.testing.assert_allclose(h[1:, 1], oh[:, 2], rtol=1e-9, atol=1e-14)


@pytest.mark.parametrize("variant", [1, 2])
def test_solve_trajectory_fp32(gpu_lib, variant):
    cfg = dict(TRAJ[1])
    tau = cfg.pop("tau")
    u0 = syn.fourier_u0(1, cfg["nx"])
    oprob, gprob = _pair(gpu_lib, dtype=torch.float32, u0=u0, **cfg)
    ref = opdhg.run(oprob, u0, tau, tau, eps=0.0, max_iter=50)
    res = gpu_lib.Solver(gprob).solve(_dev(u0, torch.float32), tau_u=tau, tau_phi=tau, eps=0.0, max_iter=50,
                                      variant=variant)
    bar_u, bar_phi = fp32_bar(oprob, u0, tau, 50, ref.u, ref.phi)
    _say(f"  bars (1e-5, or twice the FP32 emulation): u {bar_u:.3e}, phi {bar_phi:.3e}")
    assert _err(res.u, ref.u, "u") < bar_u
    assert _err(res.phi, ref.phi, "phi") < bar_phi


# ------------------------------------------------------------------ full benchmark size (2048 x 512)
BENCH = dict(nx=2048, nt=512, t_final=0.5, alpha=0.5, beta=0.0, gamma=0.0, time="bdf2", space="fd_lf")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_full_size_trajectory_matches_oracle(gpu_lib, dtype):
    """The benchmark workload in the benchmark's launch configuration, 3 iterations, every element."""
    _say(f"full-size trajectory {dtype}")
    u0 = syn.fourier_u0(0, BENCH["nx"])
    oprob, gprob = _pair(gpu_lib, dtype=dtype, u0=u0, **BENCH)
    ref = opdhg.run(oprob, u0, 0.68, 0.68, eps=0.0, max_iter=3, record=True)
    res = gpu_lib.Solver(gprob).solve(_dev(u0, dtype), tau_u=0.68, tau_phi=0.68, eps=0.0, max_iter=3,
                                      check_every=128, history=True)
    assert res.stats["variant"] == 2
    # FP32: 1e-5, or twice the error of the FP32 emulation (float storage, float FFTs and the float
    # segmented column recurrences) where the rounding amplified by 4/h_t makes that larger
    tol, tol_phi = (TOL[dtype], TOL[dtype]) if dtype == torch.float64 else \
        fp32_bar(oprob, u0, 0.68, 3, ref.u, ref.phi)
    _say(f"  tolerance u {tol:.3e}, phi {tol_phi:.3e}")
    assert _err(res.u, ref.u, "u") < tol
    assert _err(res.phi, ref.phi, "phi") < tol_phi
    np.testing.assert_allclose(res.history.cpu().numpy()[1:, 0], np.array(ref.history)[:, 1],
                               rtol=TOL[dtype] * 100)


def test_full_size_fused_equals_unfused(gpu_lib):
    """300 iterations at 2048 x 512, FP64: the fused and unfused kernels agree."""
    u0 = syn.fourier_u0(0, BENCH["nx"])
    _, gprob = _pair(gpu_lib, dtype=torch.float64, u0=u0, **BENCH)
    s = gpu_lib.Solver(gprob)
    r1 = s.solve(_dev(u0, torch.float64), tau_u=0.68, tau_phi=0.68, eps=0.0, max_iter=300, variant=1)
    u1, p1 = r1.u.clone(), r1.phi.clone()
    r2 = s.solve(_dev(u0, torch.float64), tau_u=0.68, tau_phi=0.68, eps=0.0, max_iter=300, variant=2)
    assert float((r2.u - u1).abs().max()) < 1e-11
    assert float((r2.phi - p1).abs().max()) < 1e-11 * max(1.0, float(p1.abs().max()))


def test_full_size_converges_to_newton_march(gpu_lib):
    """FP64 to residual 1e-8 at 2048 x 512: the saddle point is the BDF2 scheme's solution."""
    u0 = syn.fourier_u0(0, BENCH["nx"])
    oprob, gprob = _pair(gpu_lib, dtype=torch.float64, u0=u0, **BENCH)
    res = gpu_lib.Solver(gprob).solve(_dev(u0, torch.float64), eps=1e-8, max_iter=100000, check_every=128)
    assert res.status == 0, res.stats
    _say(f"full size converged in {res.stats['iters']} iterations, {res.stats['seconds']:.3f} s")
    nw = onewton.march(oprob, u0)
    err = float(np.max(np.abs(res.u.cpu().numpy() - nw)))
    _say(f"max |u - newton| = {err:.3e}")
    assert err < 1e-7
    m = ofd.mass(oprob, res.u.cpu().numpy())
    assert np.max(np.abs(m - m[0])) < 1e-10


# ------------------------------------------------------------------ converged solutions
def test_advection_cfl4_reaches_closed_form(gpu_lib):
    """Linear advection, 64 x 32, CFL 4, BE upwind, FP64 to 1e-10: the implicit scheme's closed form."""
    pk = gpu_lib
    u0 = syn.sine_u0(64)
    prob = pk.Problem(nx=64, nt=32, t_final=2.0, alpha=0.0, beta=1.0, time="be", space="fd_upwind",
                      dtype=torch.float64)
    res = pk.Solver(prob).solve(_dev(u0, torch.float64), tau_u=0.7, tau_phi=0.7, eps=1e-10, max_iter=5000)
    assert res.status == 0, res.stats
    assert abs(res.stats["iters"] - 1658) <= 2
    cf = advection_sine_solution(64, 32, 4.0)
    assert float(np.max(np.abs(res.u.cpu().numpy() - cf))) < 1e-10


@pytest.mark.parametrize("time", ["be", "bdf2"])
def test_burgers_converges_to_newton_march(gpu_lib, time):
    nx, nt = 128, 32
    u0 = syn.fourier_u0(0, nx)
    oprob, gprob = _pair(gpu_lib, nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.0, gamma=0.0, time=time,
                         space="fd_lf", dtype=torch.float64, u0=u0)
    res = gpu_lib.Solver(gprob).solve(_dev(u0, torch.float64), eps=1e-8, max_iter=20000)
    assert res.status == 0, res.stats
    nw = onewton.march(oprob, u0)
    assert float(np.max(np.abs(res.u.cpu().numpy() - nw))) < 2e-8
    # the GPU estimate is a Rayleigh quotient: never above nu_max, and close to it
    u_init = np.tile(u0, (nt + 1, 1))
    nm = opdhg.nu_max(oprob, u_init, iters=1500)
    assert nm * 0.99 <= res.stats["nu_max"] <= nm * (1 + 1e-9)
    assert res.stats["tau_u"] == pytest.approx(np.sqrt(0.95 / res.stats["nu_max"]), rel=1e-12)


# ------------------------------------------------------------------ adjoint
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("time", ["be", "bdf2"])
def test_adjoint_gradient_matches_oracle(gpu_lib, dtype, time):
    nx, nt = 256, 24
    u0, tgt = syn.fourier_u0(0, nx), syn.fourier_u0(1, nx)
    oprob, gprob = _pair(gpu_lib, nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.0, gamma=1e-3, time=time,
                         space="fd_lf", dtype=dtype, u0=u0)
    u = onewton.march(oprob, u0)
    g = oadj.terminal_loss_grad(oprob, u, tgt)
    ref = oadj.gradient_u0(oprob, u, g)
    mu_ref = oadj.adjoint_solve(oprob, u, g)
    solver = gpu_lib.Solver(gprob)
    grad, mu = solver.adjoint_solve(_dev(u, dtype), _dev(g, dtype), want_mu=True)
    assert _err(mu, mu_ref, "mu") < TOL[dtype]
    assert _err(grad, ref, "dl/du0") < TOL[dtype]


# ------------------------------------------------------------------ failure handling
@pytest.mark.parametrize("time", ["be", "bdf2"])
def test_lazy_dual_residual_gives_the_same_solve(gpu_lib, time):
    """Without a residual history the fused body evaluates ||J(u)^T phi|| only where ||A(u)|| <= eps or
    at max_iter; with a history, every iteration.  Iterates, n* and the reported norms agree bitwise."""
    nx, nt = 128, 32
    u0 = syn.fourier_u0(1, nx)
    _, gprob = _pair(gpu_lib, nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.0, gamma=0.0, time=time,
                     space="fd_lf", dtype=torch.float64, u0=u0)
    s = gpu_lib.Solver(gprob)
    x0 = _dev(u0, torch.float64)
    a = s.solve(x0, eps=1e-8, max_iter=20000, check_every=64)
    b = s.solve(x0, eps=1e-8, max_iter=20000, check_every=64, history=True)
    _say(f"lazy {time}: n* {a.stats['iters']} / {b.stats['iters']}")
    assert a.status == 0 and b.status == 0
    assert a.stats["iters"] == b.stats["iters"]
    assert torch.equal(a.u, b.u) and torch.equal(a.phi, b.phi)
    assert (a.stats["res_primal"], a.stats["res_dual"]) == (b.stats["res_primal"], b.stats["res_dual"])
    h = b.history.cpu().numpy()
    assert np.all(np.isfinite(h[1:]))
    # stopped by max_iter: the last iterate's dual residual is evaluated
    c = s.solve(x0, eps=1e-12, max_iter=53)
    d = s.solve(x0, eps=1e-12, max_iter=53, history=True)
    assert c.status == 1 and c.stats["iters"] == 53
    assert np.isfinite(c.stats["res_dual"]) and c.stats["res_dual"] == d.stats["res_dual"]
    assert torch.equal(c.u, d.u) and torch.equal(c.phi, d.phi)


def test_large_steps_are_detected_as_divergence(gpu_lib):
    pk = gpu_lib
    u0 = syn.sine_u0(64)
    prob = pk.Problem(nx=64, nt=32, t_final=2.0, alpha=0.0, beta=1.0, time="be", space="fd_upwind",
                      dtype=torch.float64)
    res = pk.Solver(prob).solve(_dev(u0, torch.float64), tau_u=2.0, tau_phi=2.0, eps=1e-10, max_iter=5000)
    assert res.status == 2


def test_nan_initial_data_is_detected(gpu_lib):
    pk = gpu_lib
    u0 = syn.fourier_u0(0, 64)
    u0[5] = np.nan
    prob = pk.Problem(nx=64, nt=16, t_final=0.5, alpha=0.5, beta=0.0, time="be", space="fd_lf",
                      dtype=torch.float64, lf_speed=1.0, precond_c=1.0)
    res = pk.Solver(prob).solve(_dev(u0, torch.float64), tau_u=0.6, tau_phi=0.6, eps=1e-8, max_iter=100)
    assert res.status == 2


def test_max_iter_reports_not_converged_with_stats(gpu_lib):
    pk = gpu_lib
    u0 = syn.fourier_u0(0, 64)
    prob = pk.Problem(nx=64, nt=16, t_final=0.5, alpha=0.5, beta=0.0, time="be", space="fd_lf",
                      dtype=torch.float64)
    res = pk.Solver(prob).solve(_dev(u0, torch.float64), eps=1e-12, max_iter=37)
    assert res.status == 1 and res.stats["iters"] == 37
    assert np.isfinite(res.stats["res_primal"]) and np.isfinite(res.stats["res_dual"])
