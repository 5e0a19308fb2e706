"""The allocation-free residual pdhg_residual_static (static device scratch) against pdhg_residual.

Two calls in a row on one GPU, the second on a smaller problem than the first
(the shared scratch keeps the first call's partial sums), each compared with
pdhg_residual on the same inputs: A(u) and J(u)^T phi bit for bit, the norms to
the FP64 parity bar.  A solve on a handle whose constants the static call
resolved (without factor tables) must equal the solve of a fresh handle."""
import numpy as np
import pytest
import torch

import synthetic as syn

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _inputs(nx, nt, dtype, seed, planes=None):
    rng = np.random.default_rng(seed)
    shape = (nx,) if planes is None else (planes, nx)
    u0 = syn.fourier_u0(seed, nx) if planes is None else None
    if planes is None:
        u = np.broadcast_to(u0, (nt + 1, nx)) + 0.05 * rng.standard_normal((nt + 1, nx))
        u[0] = u0
    else:
        u = 0.5 + 0.1 * rng.standard_normal((nt + 1,) + shape)
    phi = rng.standard_normal((nt,) + shape)
    dev = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")
    return dev(u), dev(phi)


CASES = [
    # the larger call first, then a smaller one
    dict(nx=4096, nt=1024, t_final=0.5, alpha=0.5, beta=0.0, time="bdf2", space="fd_lf", dtype=torch.float64),
    dict(nx=256, nt=33, t_final=0.5, alpha=0.5, beta=0.0, gamma=1e-3, time="be", space="fd_lf",
         dtype=torch.float32),
    dict(nx=64, nt=10, t_final=0.5, alpha=0.5, beta=0.0, time="be", space="dg_p2_llf", dtype=torch.float64),
]


def test_static_residual_equals_residual_on_consecutive_calls(gpu_lib):
    pk = gpu_lib
    for i, cfg in enumerate(CASES):
        cfg = dict(cfg)
        dtype = cfg["dtype"]
        _say(f"static residual call {i}: {cfg['space']} {cfg['nx']} x {cfg['nt']} {dtype}")
        planes = 3 if cfg["space"] == "dg_p2_llf" else None
        u, phi = _inputs(cfg["nx"], cfg["nt"], dtype, seed=i, planes=planes)
        a = pk.Solver(pk.Problem(**cfg))
        b = pk.Solver(pk.Problem(**cfg))
        au_ref, jt_ref, res_ref = a.residual(u, phi)
        au = torch.full_like(au_ref, float("nan"))
        jt = torch.full_like(jt_ref, float("nan"))
        _, _, res = b.residual_static(u, phi, au, jt)
        torch.cuda.synchronize()
        assert torch.equal(au, au_ref), "A(u) differs"
        assert torch.equal(jt, jt_ref), "J^T phi differs"
        for k in range(2):
            _say(f"  norm {k}: {res[k]:.17e} vs {res_ref[k]:.17e}")
            assert res[k] == pytest.approx(res_ref[k], rel=1e-12)
        # norms only (no fields), and without phi
        _, _, res2 = b.residual_static(u, None, None, None)
        assert res2[0] == pytest.approx(res_ref[0], rel=1e-12) and res2[1] == 0.0


def test_solve_after_static_residual_is_unchanged(gpu_lib):
    """The static call resolves the default constants without building the factor tables; a later
    solve on that handle builds them and runs exactly as on a fresh handle."""
    pk = gpu_lib
    cfg = dict(nx=512, nt=64, t_final=0.5, alpha=0.5, beta=0.0, time="bdf2", space="fd_lf", dtype=torch.float64)
    u0 = torch.tensor(syn.fourier_u0(3, 512), dtype=torch.float64, device="cuda")
    u = u0.repeat(65, 1).contiguous()
    s1 = pk.Solver(pk.Problem(**cfg))
    s1.residual_static(u)
    r1 = s1.solve(u0, tau_u=0.6, tau_phi=0.6, eps=0.0, max_iter=20)
    u1, p1 = r1.u.clone(), r1.phi.clone()
    r2 = pk.Solver(pk.Problem(**cfg)).solve(u0, tau_u=0.6, tau_phi=0.6, eps=0.0, max_iter=20)
    assert torch.equal(u1, r2.u) and torch.equal(p1, r2.phi)
