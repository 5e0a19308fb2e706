"""Differentiable solve (viscous Burgers, backward Euler, Lax-Friedrichs + centred
diffusion): the autograd gradient d loss / d u0 through the implicit adjoint,
against the FP64 oracle gradient and FP64 central finite differences."""
import numpy as np
import pytest
import torch

import synthetic as syn
from oracle import adjoint as oadj
from oracle import newton as onewton
from oracle.problem import Problem as OProblem, default_constants

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _setup(pk, nx, nt, dtype):
    u0 = syn.fourier_u0(0, nx)
    tgt = syn.fourier_u0(1, nx)
    oprob = default_constants(OProblem(nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.0, gamma=1e-3,
                                       space="fd_lf", time="be"), u0)
    gprob = pk.Problem(nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.0, gamma=1e-3, time="be", space="fd_lf",
                       dtype=dtype, lf_speed=oprob.lf_speed, precond_c=oprob.precond_c,
                       precond_gamma_hat=1e-3)
    return u0, tgt, oprob, gprob


def _loss_torch(u, tgt, hx):
    d = u[-1] - tgt
    return hx * (d * d).sum()


def _gpu_grad(pk, gprob, u0, tgt, eps, max_iter, **kw):
    dev = "cuda"
    solver = pk.Solver(gprob)
    x = torch.tensor(u0, dtype=gprob.torch_dtype, device=dev, requires_grad=True)
    t = torch.tensor(tgt, dtype=gprob.torch_dtype, device=dev)
    u = pk.differentiable_solve(x, solver, eps=eps, max_iter=max_iter, check_every=128, **kw)
    loss = _loss_torch(u, t, 1.0 / gprob.nx)
    loss.backward()
    return x.grad.detach().cpu().double().numpy(), u.detach().cpu().double().numpy(), float(loss)


def test_full_size_gradient_matches_oracle_fp64(gpu_lib):
    nx, nt = 2048, 512
    u0, tgt, oprob, gprob = _setup(gpu_lib, nx, nt, torch.float64)
    g, u, loss = _gpu_grad(gpu_lib, gprob, u0, tgt, eps=1e-10, max_iter=200000)
    nw = onewton.march(oprob, u0)
    _say(f"max |u - newton| = {np.max(np.abs(u - nw)):.3e}")
    ref = oadj.gradient_u0(oprob, nw, oadj.terminal_loss_grad(oprob, nw, tgt))
    err = np.max(np.abs(g - ref)) / np.max(np.abs(ref))
    _say(f"gradient rel err vs oracle: {err:.3e}")
    assert err < 1e-8
    assert loss == pytest.approx(oadj.terminal_loss(oprob, nw, tgt), rel=1e-9)
    # central differences of the oracle's Newton march on 16 unit directions (h = 1e-6)
    for d in syn.unit_directions(2, nx, 16):
        h = 1e-6
        lp = oadj.terminal_loss(oprob, onewton.march(oprob, u0 + h * d), tgt)
        lm = oadj.terminal_loss(oprob, onewton.march(oprob, u0 - h * d), tgt)
        fdv = (lp - lm) / (2 * h)
        _say(f"  direction: FD {fdv:.10e} adjoint {g @ d:.10e}")
        assert abs(fdv - g @ d) <= 1e-6 * max(abs(fdv), 1e-8) + 1e-11


def test_gradient_matches_central_differences_16_directions(gpu_lib):
    nx, nt = 512, 128
    u0, tgt, oprob, gprob = _setup(gpu_lib, nx, nt, torch.float64)
    g, _, _ = _gpu_grad(gpu_lib, gprob, u0, tgt, eps=1e-11, max_iter=100000)
    for d in syn.unit_directions(2, nx, 16):
        h = 1e-6
        lp = oadj.terminal_loss(oprob, onewton.march(oprob, u0 + h * d), tgt)
        lm = oadj.terminal_loss(oprob, onewton.march(oprob, u0 - h * d), tgt)
        fdv = (lp - lm) / (2 * h)
        assert abs(fdv - g @ d) <= 1e-6 * max(abs(fdv), 1e-8) + 1e-11, (fdv, g @ d)


def test_fp32_adjoint_kernel_at_full_size(gpu_lib):
    """The FP32 adjoint march on the FP64 solution (rounded to FP32) against the FP64 oracle gradient."""
    nx, nt = 2048, 512
    u0, tgt, oprob, gprob = _setup(gpu_lib, nx, nt, torch.float32)
    nw = onewton.march(oprob, u0)
    gl = oadj.terminal_loss_grad(oprob, nw, tgt)
    ref = oadj.gradient_u0(oprob, nw, gl)
    solver = gpu_lib.Solver(gprob)
    g = solver.adjoint_solve(torch.tensor(nw, dtype=torch.float32, device="cuda"),
                             torch.tensor(gl, dtype=torch.float32, device="cuda"))
    err = float(np.max(np.abs(g.cpu().double().numpy() - ref)) / np.max(np.abs(ref)))
    _say(f"FP32 adjoint rel err: {err:.3e}")
    assert err < 1e-5


def test_fp32_pipeline_gradient(gpu_lib):
    """FP32 solve (to its stop rule) + FP32 adjoint: reported error against FP64, bounded by the
    FP32 solution error propagated through the loss (the gradient inherits |u32 - u64| / |u|)."""
    nx, nt = 2048, 512
    u0, tgt, oprob, gprob = _setup(gpu_lib, nx, nt, torch.float32)
    # to the FP32 rounding floor: stop when ||A(u)|| has not improved for 1000 iterations (the scale-free
    # tolerance 1e-6 ||u0|| / h_t stops earlier, at max |u - newton| ~3e-4 on this grid)
    g, u, _ = _gpu_grad(gpu_lib, gprob, u0, tgt, eps=1e-8, max_iter=100000, stall_iters=1000)
    nw = onewton.march(oprob, u0)
    ref = oadj.gradient_u0(oprob, nw, oadj.terminal_loss_grad(oprob, nw, tgt))
    uerr = float(np.max(np.abs(u - nw)))
    gerr = float(np.max(np.abs(g - ref)) / np.max(np.abs(ref)))
    _say(f"FP32 pipeline: max|u - newton| = {uerr:.3e}, gradient rel err {gerr:.3e}")
    assert gerr < 1e-5


def test_unconverged_forward_is_refused(gpu_lib):
    """The implicit adjoint holds at A(u) = 0: a forward solve stopped by max_iter raises, unless the
    caller accepts it explicitly (then a warning names the residual)."""
    nx, nt = 128, 32
    u0, tgt, oprob, gprob = _setup(gpu_lib, nx, nt, torch.float64)
    with pytest.raises(RuntimeError, match="max_iter"):
        _gpu_grad(gpu_lib, gprob, u0, tgt, eps=1e-10, max_iter=20)
    with pytest.warns(RuntimeWarning, match="max_iter"):
        g, _, _ = _gpu_grad(gpu_lib, gprob, u0, tgt, eps=1e-10, max_iter=20, allow_unconverged=True)
    assert np.all(np.isfinite(g))
