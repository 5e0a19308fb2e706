"""Batched solver: every problem of a batch follows the iterates of its own
single-problem solve (which the other GPU tests pin to the oracle), and small
batches are checked against the FP64 oracle directly."""
import numpy as np
import pytest
import torch

import synthetic as syn
from oracle import newton as onewton
from oracle import pdhg as opdhg
from oracle.problem import Problem as OProblem, default_constants

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _rel(a, b):
    a = a.detach().cpu().double().numpy() if torch.is_tensor(a) else np.asarray(a)
    b = b.detach().cpu().double().numpy() if torch.is_tensor(b) else np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(1.0, np.max(np.abs(b))))


# A mixed batch: uneven nx and nt (odd nt included), both time schemes, both
# fluxes, viscous and inviscid, linear and Burgers.  Algorithm 1 converges on
# each of them (checked with the oracle); for nonlinear laws it need not
# (Section 3.3 makes no convergence claim there), see the 256-problem test.
MIXED = [
    dict(nx=256, nt=64, t_final=0.5, alpha=0.5, beta=0.0, gamma=0.0, time="bdf2", space="fd_lf", seed=0),
    dict(nx=512, nt=33, t_final=0.125, alpha=0.5, beta=0.0, gamma=1e-3, time="be", space="fd_lf", seed=2),
    dict(nx=1024, nt=64, t_final=1.0, alpha=0.0, beta=1.0, gamma=0.0, time="be", space="fd_upwind", seed=3),
    dict(nx=256, nt=7, t_final=0.05, alpha=0.5, beta=0.0, gamma=0.0, time="bdf2", space="fd_lf", seed=4),
    dict(nx=2048, nt=40, t_final=0.05, alpha=0.5, beta=0.0, gamma=0.0, time="bdf2", space="fd_lf", seed=0),
    dict(nx=4096, nt=24, t_final=0.02, alpha=0.5, beta=0.0, gamma=5e-4, time="bdf2", space="fd_lf", seed=6),
    dict(nx=256, nt=16, t_final=0.125, alpha=0.5, beta=0.0, gamma=0.0, time="bdf2", space="fd_lf", seed=1),
]


def _problems(pk, cfgs, dtype):
    probs, u0s = [], []
    for c in cfgs:
        c = dict(c)
        seed = c.pop("seed")
        probs.append(pk.Problem(dtype=dtype, **c))
        u0s.append(syn.fourier_u0(seed, c["nx"]))
    return probs, u0s


def _single(pk, prob, u0, tau, n_iter, eps=0.0, check_every=8):
    s = pk.Solver(prob)
    r = s.solve(torch.tensor(u0, dtype=prob.torch_dtype, device="cuda"), tau_u=tau, tau_phi=tau, eps=eps,
                max_iter=n_iter, check_every=check_every, variant=2)
    return r


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_mixed_batch_follows_single_solves(gpu_lib, dtype):
    pk = gpu_lib
    probs, u0s = _problems(pk, MIXED, dtype)
    bs = pk.BatchSolver(probs)
    u0 = bs.pack_u0(u0s)
    n_iter = 60
    _say(f"mixed batch {dtype}: {len(probs)} problems, {n_iter} iterations")
    res = bs.solve(u0, eps=0.0, max_iter=n_iter, check_every=8)
    assert res.status == 1
    for i, (p, x0) in enumerate(zip(probs, u0s)):
        st = res.stats[i]
        assert st["iters"] == n_iter and st["status"] == 1
        ref = _single(pk, p, x0, st["tau_u"], n_iter)
        assert ref.stats["tau_u"] == st["tau_u"]
        eu, ep = _rel(res.views_u[i], ref.u), _rel(res.views_phi[i], ref.phi)
        _say(f"  problem {i} nx={p.nx} nt={p.nt}: |u - single| {eu:.2e}  |phi - single| {ep:.2e}  "
             f"Rp {st['res_primal']:.4e} vs {ref.stats['res_primal']:.4e}")
        tol = 1e-12 if dtype == torch.float64 else 1e-6
        assert eu <= tol and ep <= tol
        assert st["res_primal"] == pytest.approx(ref.stats["res_primal"], rel=1e-9 if dtype == torch.float64 else 1e-4)
        assert st["res_dual"] == pytest.approx(ref.stats["res_dual"], rel=1e-9 if dtype == torch.float64 else 1e-4)


def test_small_batch_matches_oracle_trajectory(gpu_lib):
    """Two problems, FP64: the batch iterate after 40 iterations against the oracle's Algorithm 1."""
    pk = gpu_lib
    cfgs = [MIXED[0], MIXED[3]]
    probs, u0s = _problems(pk, cfgs, torch.float64)
    bs = pk.BatchSolver(probs)
    tau = [0.6, 0.55]
    res = bs.solve(bs.pack_u0(u0s), tau_u=tau, tau_phi=tau, eps=0.0, max_iter=40, check_every=4)
    for i, c in enumerate(cfgs):
        c = {k: v for k, v in c.items() if k != "seed"}
        op = default_constants(OProblem(**c), u0s[i])
        ref = opdhg.run(op, u0s[i], tau[i], tau[i], eps=0.0, max_iter=40)
        eu, ep = _rel(res.views_u[i], ref.u), _rel(res.views_phi[i], ref.phi)
        _say(f"  problem {i}: |u - oracle| {eu:.2e}  |phi - oracle| {ep:.2e}")
        assert eu < 1e-10 and ep < 1e-10


def test_batch_converges_per_problem(gpu_lib):
    """FP64 to residual 1e-8: each problem stops at its own n*, equal to its single solve's, and the
    converged u agrees with the oracle's Newton march of the implicit scheme."""
    pk = gpu_lib
    cfgs = [MIXED[0], MIXED[1], MIXED[3], MIXED[6]]
    probs, u0s = _problems(pk, cfgs, torch.float64)
    bs = pk.BatchSolver(probs)
    res = bs.solve(bs.pack_u0(u0s), eps=1e-8, max_iter=50000, check_every=32)
    assert res.status == 0
    for i, c in enumerate(cfgs):
        st = res.stats[i]
        ref = _single(pk, probs[i], u0s[i], st["tau_u"], 50000, eps=1e-8)
        c = {k: v for k, v in c.items() if k != "seed"}
        op = default_constants(OProblem(**c), u0s[i])
        nw = onewton.march(op, u0s[i])
        en = float(np.max(np.abs(res.views_u[i].cpu().numpy() - nw)))
        _say(f"  problem {i}: n* {st['iters']} (single {ref.stats['iters']}), |u - newton| {en:.2e}, "
             f"mass drift {st['mass_drift']:.2e}")
        assert st["status"] == 0
        assert st["iters"] == ref.stats["iters"]
        assert max(st["res_primal"], st["res_dual"]) <= 1e-8
        assert en < 1e-6
        assert st["mass_drift"] < 1e-8   # |m^l - m^0| <= T ||A(u)|| up to norm constants


def test_autotuned_grids_do_not_change_results(gpu_lib):
    pk = gpu_lib
    probs, u0s = _problems(pk, MIXED, torch.float32)
    bs = pk.BatchSolver(probs)
    u0 = bs.pack_u0(u0s)
    a = bs.solve(u0, eps=0.0, max_iter=30, check_every=6)
    ua, pa = a.u.clone(), a.phi.clone()
    taus = [s["tau_u"] for s in a.stats]
    grids = bs.tune(u0, tau_u=taus, tau_phi=taus)
    _say(f"  tuned grids {grids}")
    assert all(g >= 1 for g in grids)
    b = bs.solve(u0, tau_u=taus, tau_phi=taus, eps=0.0, max_iter=30, check_every=6)
    assert torch.equal(ua, b.u) and torch.equal(pa, b.phi)


def test_warm_start_from_converged_batch(gpu_lib):
    pk = gpu_lib
    cfgs = [MIXED[0], MIXED[3]]
    probs, u0s = _problems(pk, cfgs, torch.float64)
    bs = pk.BatchSolver(probs)
    u0 = bs.pack_u0(u0s)
    a = bs.solve(u0, eps=1e-9, max_iter=50000, check_every=16)
    taus = [s["tau_u"] for s in a.stats]
    b = bs.solve(u0, tau_u=taus, tau_phi=taus, eps=2e-9, max_iter=50000, check_every=16, u=a.u.clone(),
                 phi=a.phi.clone(), warm_start=True)
    for s in b.stats:
        assert s["status"] == 0 and s["iters"] <= 1


def test_256_burgers_batch_sampled_against_single_solves(gpu_lib):
    """256 Burgers problems (BDF2, LF, T = 0.5), nx in {256..4096}, nt in {64..512}, FP32, 150
    iterations.  Algorithm 1 diverges on some of these initial data (the saddle problem of a nonlinear
    law is not convex); a diverged problem stops and drops out of the batch.  Eight sampled problems
    (the largest and smallest among them) end with the status, n* and iterates of their single solves."""
    pk = gpu_lib
    shapes = syn.batch_shapes(0, 256)
    probs = [pk.Problem(nx=nx, nt=nt, t_final=0.5, alpha=0.5, beta=0.0, time="bdf2", space="fd_lf",
                        dtype=torch.float32) for nx, nt, _ in shapes]
    u0s = [syn.fourier_u0(s, nx) for nx, _, s in shapes]
    bs = pk.BatchSolver(probs)
    _say(f"256-problem batch: {sum((p.nt + 1) * p.nx for p in probs)} u points")
    res = bs.solve(bs.pack_u0(u0s), eps=0.0, max_iter=150, check_every=50)
    nd = sum(s["status"] == 2 for s in res.stats)
    _say(f"  {nd} of 256 diverged within 150 iterations")
    assert res.status in (1, 2)
    assert all(s["status"] in (1, 2) for s in res.stats)
    size = [p.nx * p.nt for p in probs]
    pick = sorted(set([int(np.argmax(size)), int(np.argmin(size))] + list(range(0, 256, 43))))
    for i in pick:
        st = res.stats[i]
        # the same chunk length, so that a diverged problem returns the same last good checkpoint
        ref = _single(pk, probs[i], u0s[i], st["tau_u"], 150, check_every=50)
        assert (st["status"], st["iters"]) == (ref.stats["status"], ref.stats["iters"])
        eu, ep = _rel(res.views_u[i], ref.u), _rel(res.views_phi[i], ref.phi)
        what = "max_iter" if st["status"] == 1 else "diverged; checkpoint"
        _say(f"  problem {i} nx={probs[i].nx} nt={probs[i].nt}: {what} n* = {st['iters']}, |u - single| {eu:.2e} "
             f"|phi - single| {ep:.2e}")
        assert eu <= 1e-6 and ep <= 1e-6
        if st["status"] == 2:
            assert st["res_primal"] == pytest.approx(ref.stats["res_primal"], rel=1e-6)
