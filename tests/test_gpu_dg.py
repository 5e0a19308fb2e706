"""DG P2 / local Lax-Friedrichs path on the GPU against the FP64 oracle (oracle/dg.py)."""
import numpy as np
import pytest
import torch

import synthetic as syn
from oracle import dg as odg
from oracle import newton as onewton
from oracle import pdhg as opdhg
from oracle.problem import Problem as OProblem, default_constants

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-10, torch.float32: 1e-5}


def _say(msg):
    print(msg, flush=True)


def _err(gpu, ref, name=""):
    g = gpu.detach().cpu().double().numpy()
    e = float(np.max(np.abs(g - ref)) / max(1.0, np.max(np.abs(ref))))
    _say(f"  rel err {name}: {e:.3e}")
    return e


def _case(pk, nx, nt, time, dtype, t_final=None, seed=0, c=None):
    u0 = odg.p2_project(lambda x: syn.fourier_u0_at(seed, x), nx)
    T = 3.0 * nt / nx if t_final is None else t_final      # h_t = 3 h_x
    op = OProblem(nx=nx, nt=nt, t_final=T, alpha=0.5, beta=0.0, space="dg_p2_llf", time=time,
                  precond_c=0.0 if c is None else c)
    op = default_constants(op, u0)
    gp = pk.Problem(nx=nx, nt=nt, t_final=T, alpha=0.5, beta=0.0, space="dg_p2_llf", time=time, dtype=dtype,
                    precond_c=-1.0 if c is None else c)
    return u0, op, gp


def _dev(x, dtype):
    return torch.tensor(np.asarray(x), dtype=dtype, device="cuda")


CASES = [(16, 5, "be"), (64, 12, "bdf2"), (256, 7, "be"), (128, 70, "bdf2")]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nx,nt,time", CASES)
def test_residual_and_dual_operator_match_oracle(gpu_lib, dtype, nx, nt, time):
    u0, op, gp = _case(gpu_lib, nx, nt, time, dtype)
    rng = np.random.default_rng(7)
    u = np.broadcast_to(u0, (nt + 1, 3, nx)) + 0.05 * rng.standard_normal((nt + 1, 3, nx))
    u[0] = u0
    phi = rng.standard_normal((nt, 3, nx))
    s = gpu_lib.Solver(gp)
    au, jt, res = s.residual(_dev(u, dtype), _dev(phi, dtype))
    ra = odg.p2_residual(op, u)
    rj = odg.p2_apply_jt(op, u, phi)
    assert _err(au, ra, "A(u)") < TOL[dtype]
    assert _err(jt, rj, "J^T phi") < TOL[dtype]
    assert res[0] == pytest.approx(odg.p2_wnorm(op, ra), rel=1e-9 if dtype == torch.float64 else 1e-5)
    jt2 = s.apply_jt(_dev(u, dtype), _dev(phi, dtype))
    assert _err(jt2, rj, "J^T phi (adjoint apply)") < TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nx,nt,time", CASES[:3] + [(32, 200, "be")])
def test_precond_matches_oracle(gpu_lib, dtype, nx, nt, time):
    u0, op, gp = _case(gpu_lib, nx, nt, time, dtype, c=0.8)
    r = np.random.default_rng(8).standard_normal((nt, 3, nx))
    s = gpu_lib.Solver(gp)
    out = s.precond(_dev(r, dtype))
    ref = odg.p2_kd_solve(op, r)
    assert _err(out, ref, "K_d^-1 r") < (1e-10 if dtype == torch.float64 else 1e-5)


@pytest.mark.parametrize("n_iter", [1, 10, 100])
@pytest.mark.parametrize("nx,nt,time", [(16, 6, "be"), (32, 8, "bdf2"), (64, 10, "be"), (128, 9, "bdf2")])
def test_trajectory_matches_oracle_fp64(gpu_lib, nx, nt, time, n_iter):
    u0, op, gp = _case(gpu_lib, nx, nt, time, torch.float64)
    tau = 0.6
    ref = opdhg.run(op, u0, tau, tau, eps=0.0, max_iter=n_iter, record=True)
    s = gpu_lib.Solver(gp)
    res = s.solve(_dev(u0, torch.float64), tau_u=tau, tau_phi=tau, eps=0.0, max_iter=n_iter, check_every=4,
                  history=True)
    assert res.stats["iters"] == n_iter and res.stats["variant"] == 4
    assert _err(res.u, ref.u, "u") < 1e-10
    assert _err(res.phi, ref.phi, "phi") < 1e-10
    h = res.history.cpu().numpy()
    oh = np.array(ref.history)
    np.testing.assert_allclose(h[1:, 0], oh[:, 1], rtol=1e-9)
    np.testing.assert_allclose(h[1:, 1], oh[:, 2], rtol=1e-9, atol=1e-14)


def test_trajectory_fp32(gpu_lib):
    u0, op, gp = _case(gpu_lib, 32, 8, "bdf2", torch.float32)
    tau, n = 0.6, 30
    ref = opdhg.run(op, u0, tau, tau, eps=0.0, max_iter=n)
    res = gpu_lib.Solver(gp).solve(_dev(u0, torch.float32), tau_u=tau, tau_phi=tau, eps=0.0, max_iter=n,
                                   check_every=4)
    # FP32 rounding of phibar amplified by tau times the row sum of |J^T| (about 4/h_t + 2 max|f'| 25/h_x
    # for the P2 coefficients), over n iterations
    row = 4.0 / op.ht + 2.0 * 25.0 * max(op.precond_c, 1.0) / op.hx
    tol = 4.0 * n * float(np.finfo(np.float32).eps) * tau * row * 2.0 * float(np.max(np.abs(ref.phi))) + 1e-5
    _say(f"  FP32 trajectory bound {tol:.2e}")
    assert _err(res.u, ref.u, "u") < tol
    assert _err(res.phi, ref.phi, "phi") < tol


def test_converges_to_newton_march_with_conserved_cell_averages(gpu_lib):
    u0, op, gp = _case(gpu_lib, 32, 8, "be", torch.float64)
    res = gpu_lib.Solver(gp).solve(_dev(u0, torch.float64), eps=1e-10, max_iter=50000, check_every=32)
    nw = onewton.march(op, u0)
    _say(f"  n* {res.stats['iters']}, tau {res.stats['tau_u']:.4f}, mass drift {res.stats['mass_drift']:.2e}")
    assert res.status == 0
    assert _err(res.u, nw, "u - newton") < 1e-8
    assert res.stats["mass_drift"] < 1e-9
    tu, _, nu = opdhg.auto_steps(op, u0, iters=1500)
    assert res.stats["nu_max"] <= nu * (1 + 1e-9) and res.stats["nu_max"] >= 0.99 * nu


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_full_size_first_iterate_sampled_modes(gpu_lib, dtype):
    """4096 cells x 512 levels, h_t = 3 h_x, backward Euler.  From u^l = u0, phi = 0, one iteration
    leaves u unchanged and sets phi = tau K_d^{-1} r with every row r^l = F(u0).  For sampled Fourier
    modes m, the DFT over the cells of GPU phi / tau must equal the oracle's per-mode solve."""
    nx, nt = 4096, 512
    u0, op, gp = _case(gpu_lib, nx, nt, "be", dtype)
    tau = 0.5
    s = gpu_lib.Solver(gp)
    res = s.solve(_dev(u0, dtype), tau_u=tau, tau_phi=tau, eps=0.0, max_iter=1, check_every=2)
    phi = res.phi.detach().cpu().double().numpy() / tau             # (nt, 3, nx)
    F = odg.spatial_operator(op, u0)                                  # (3, nx), the same on every row
    Fh = np.fft.fft(F, axis=-1)
    b = np.zeros((nt, nt))
    for l in range(nt):
        b[l, l] = 1.0 / op.ht
        if l >= 1:
            b[l, l - 1] = -1.0 / op.ht
    kt = b @ b.T
    worst = 0.0
    spec = np.fft.fft(phi, axis=-1)
    scale = float(np.max(np.abs(spec)))          # errors relative to the spectrum's scale (most modes ~0)
    for m in (0, 1, 2, 3, 7, 513, 2048):
        g = odg.symbol(op, 2 * np.pi * m / nx)
        w, q = np.linalg.eigh(op.precond_c ** 2 * (g @ g.conj().T))
        rhs = np.tile(Fh[:, m], (nt, 1)) @ q.conj()                   # (nt, 3)
        z = np.stack([np.linalg.solve(kt + w[k] * np.eye(nt), rhs[:, k]) for k in range(3)], axis=1)
        ref = z @ q.T                                                 # (nt, 3)
        got = spec[:, :, m]
        e = float(np.max(np.abs(got - ref)) / scale)
        worst = max(worst, e)
        _say(f"  mode {m}: rel err {e:.3e}")
    assert np.array_equal(res.u.detach().cpu().double().numpy()[1:], np.broadcast_to(u0, (nt, 3, nx)).astype(
        np.float32 if dtype == torch.float32 else np.float64).astype(np.float64))
    assert worst < (1e-10 if dtype == torch.float64 else 1e-5)


def test_full_size_fp32_tracks_fp64(gpu_lib):
    """4096 x 512: 50 iterations in FP32 against FP64 with the same step sizes (rounding bound)."""
    nx, nt = 4096, 512
    u0, op, gp64 = _case(gpu_lib, nx, nt, "be", torch.float64)
    _, _, gp32 = _case(gpu_lib, nx, nt, "be", torch.float32)
    r64 = gpu_lib.Solver(gp64).solve(_dev(u0, torch.float64), eps=0.0, max_iter=50, check_every=10)
    tau = r64.stats["tau_u"]
    r32 = gpu_lib.Solver(gp32).solve(_dev(u0, torch.float32), tau_u=tau, tau_phi=tau, eps=0.0, max_iter=50,
                                     check_every=10)
    u64 = r64.u.cpu().numpy()
    e = _err(r32.u, u64, "u FP32 vs FP64")
    row = 4.0 / op.ht + 2.0 * 25.0 * max(op.precond_c, 1.0) / op.hx
    tol = 4.0 * 50 * float(np.finfo(np.float32).eps) * tau * row * 2.0 * float(r64.phi.abs().max()) + 1e-5
    _say(f"  bound {tol:.2e}; tau {tau:.4f}")
    assert e < tol
