"""CPU primal-dual iteration (Algorithm 1, Section 3.3) -- oracle, test infrastructure only.

Algorithm 1 with the initial level held fixed (u^0 = u0; the lambda
multiplier of Section 3.3 is not used, see the readings below) and the
standard PDHG signs of Section 2.2:

    start:  u^l = u0 for all l,  phi = 0,  phibar = 0            (Section 3.3)
    repeat
        u     <- u - tau_u J(u)^T phibar        (primal step, Section 2.2; J at
                                                 the current iterate)
        r     <- A(u)                           (implicit residual at the new u)
        s     <- K_d^{-1} r                     (dual proximal step in ||.||_H)
        phibar <- phi + 2 tau_phi s ;  phi <- phi + tau_phi s     (extrapolation)
        Res    = [ ||A(u)||, ||J(u)^T phi|| ]   (Section 2.3, space-time L2 norm)
    until both entries of Res <= eps  or  n = max_iter

Readings: the printed Algorithm 1 flips the sign of both the primal and the
dual step relative to its Lagrangian; this is the same iteration under
phi -> -phi, so the u iterates coincide.  The lambda variant is not used:
its boundary terms carry inconsistent signs.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import fd
from .precond import kd_solve
from .problem import Problem


@dataclass
class PdhgResult:
    u: np.ndarray                 # (N_t+1, N_x) including u^0
    phi: np.ndarray               # (N_t, N_x)
    iters: int
    res_primal: float
    res_dual: float
    converged: bool
    history: list = field(default_factory=list)   # [(n, Rp, Rd)]


def _ops(prob: Problem):
    """Residual / J^T / norm functions for the problem's discretisation."""
    if prob.space == "dg_p2_llf":
        from . import dg
        return dg.p2_residual, dg.p2_apply_jt, dg.p2_wnorm
    if prob.space == "dg_p1_upwind":
        from . import dg1
        return dg1.p1_residual, dg1.p1_apply_jt, dg1.p1_wnorm
    return fd.residual, fd.apply_jt, fd.wnorm


def run(prob: Problem, u0: np.ndarray, tau_u: float, tau_phi: float, eps: float = 0.0,
        max_iter: int = 1000, u_init=None, phi_init=None, record: bool = False) -> PdhgResult:
    """Run Algorithm 1 (u^0 fixed) and return the iterate at the stopping index n*.

    The residual is evaluated after every iteration; the loop stops at the
    first n with max(Rp, Rd) <= eps.  eps = 0 runs exactly max_iter
    iterations.  With warm-start arrays, phibar starts equal to phi.
    """
    residual, apply_jt, wnorm = _ops(prob)
    shape_u = (prob.nt + 1,) + np.shape(u0)
    if u_init is None:
        u = np.broadcast_to(np.asarray(u0, dtype=np.float64), shape_u).copy()
    else:
        u = np.array(u_init, dtype=np.float64)
        u[0] = u0
    phi = np.zeros((prob.nt,) + np.shape(u0)) if phi_init is None else np.array(phi_init, dtype=np.float64)
    phibar = phi.copy()
    hist = []
    rp = rd = float("inf")
    n = 0
    # J(u^n)^T is needed twice: for the dual residual of iterate n and for the
    # primal step of iteration n+1; both use the same u^n.
    jt = jt_operator(prob, u)
    for n in range(1, max_iter + 1):
        u[1:] -= tau_u * jt(phibar)
        r = residual(prob, u)
        s = kd_solve_any(prob, r)
        phibar = phi + 2.0 * tau_phi * s
        phi = phi + tau_phi * s
        jt = jt_operator(prob, u)
        rp = wnorm(prob, r)
        rd = wnorm(prob, jt(phi))
        if record:
            hist.append((n, rp, rd))
        if not (np.isfinite(rp) and np.isfinite(rd)):
            break
        if max(rp, rd) <= eps:
            return PdhgResult(u, phi, n, rp, rd, True, hist)
    return PdhgResult(u, phi, n, rp, rd, False, hist)


def jt_operator(prob: Problem, u: np.ndarray):
    """phi -> J(u)^T phi with J assembled once at u."""
    if prob.space == "dg_p2_llf":
        from . import dg
        return lambda phi: dg.p2_apply_jt(prob, u, phi)
    if prob.space == "dg_p1_upwind":
        from . import dg1
        jt = dg1.p1_jacobian(prob, u).T.tocsr()
        return lambda phi: (jt @ phi.ravel()).reshape(phi.shape)
    jt = fd.jacobian(prob, u).T.tocsr()
    return lambda phi: (jt @ phi.ravel()).reshape(phi.shape)


def kd_solve_any(prob: Problem, r: np.ndarray) -> np.ndarray:
    if prob.space == "dg_p2_llf":
        from . import dg
        return dg.p2_kd_solve(prob, r)
    if prob.space == "dg_p1_upwind":
        from . import dg1
        return dg1.p1_kd_solve(prob, r)
    if prob.precond_kind == "full":
        from .precond import kd_full_solve
        return kd_full_solve(prob, r)
    return kd_solve(prob, r)


def nu_max(prob: Problem, u: np.ndarray, iters: int = 200, seed: int = 0) -> float:
    """Largest eigenvalue of J(u)^T K_d^{-1} J(u) by power iteration.

    Proposition 2.1 requires sigma * tau * nu < 1 for every eigenvalue nu.
    """
    residual, apply_jt, _ = _ops(prob)
    if prob.space == "dg_p1_upwind":
        from . import dg1
        J = dg1.p1_jacobian(prob, u)
    else:
        J = fd.jacobian(prob, u) if prob.space != "dg_p2_llf" else None
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((prob.nt,) + np.shape(u[0]))
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        if J is not None:
            w = (J @ v.ravel()).reshape(v.shape)
            w = kd_solve_any(prob, w)
            w = (J.T @ w.ravel()).reshape(v.shape)
        else:
            from . import dg
            w = dg.p2_apply_j(prob, u, v)
            w = kd_solve_any(prob, w)
            w = apply_jt(prob, u, w)
        lam = float(np.sum(w * v))
        v = w / np.linalg.norm(w)
    return lam


def auto_steps(prob: Problem, u0: np.ndarray, safety: float = 0.95, iters: int = 200):
    """sigma = tau = sqrt(safety / nu_max) at the initial guess u^l = u0."""
    u = np.broadcast_to(np.asarray(u0, dtype=np.float64), (prob.nt + 1,) + np.shape(u0)).copy()
    nm = nu_max(prob, u, iters)
    t = float(np.sqrt(safety / nm))
    return t, t, nm
