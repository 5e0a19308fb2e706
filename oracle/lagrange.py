"""Algorithm 1 with the initial level as an unknown and a multiplier for it (Section 3.3) -- oracle, test
infrastructure only.

Section 3.3 adds a dual variable lambda_j that imposes the initial condition, so
that u^0 becomes an unknown of the saddle problem:

    L(u, phi, lambda) = h_t h_x sum_{l, j} phi^l_j A(u)^l_j  +  h_x sum_j lambda_j (u^0_j - u0_j),

with A the implicit residual of Sections 3.1-3.2, whose rows 0 (and 1 for BDF2) now
depend on the unknown u^0 through their time differences.  The printed algorithm
takes both dual steps with inconsistent signs (the phi step is written as a descent,
the lambda step as an ascent, and the boundary term of the rewritten Lagrangian
carries the opposite sign), and it leaves tau_{u0} undefined.  Reading used here:
standard primal-dual steps on L (descent in u, ascent in phi and lambda), each block
measured in its own weight in L (h_t h_x for u^l and phi, h_x for u^0 and lambda):

    u^l    <- u^l - tau_u (J(u)^T phibar)^l                          l = 1..N_t
    u^0    <- u^0 - tau_u0 ( h_t (J_0^T phibar) + lambdabar )         J_0 = dA/du^0
    phi    <- phi + tau_phi K_d^{-1} A(u);      phibar    = 2 phi_new - phi_old
    lambda <- lambda + tau_lam (u^0 - u0);      lambdabar = 2 lambda_new - lambda_old

J_0 acts through the time differences only: row 0 holds c1/h_t (backward Euler,
c1 = -1) and, for BDF2, row 1 holds c2/h_t (c2 = 1/2), so
h_t J_0^T phi = c1 phi^0 + c2 phi^1 point by point, for finite differences and for
the DG nodal values alike.  tau_u0 defaults to tau_u / 2: the paper leaves it
undefined, and the u^0 block couples to lambda (an identity) on top of its coupling
to phi, so the full primal step there can break the joint step condition (the CFL-4
advection case diverges with tau_u0 = tau_u = 0.7 and converges with 0.35).  The
stopping test is the
paper's Res(u, phi) = [||A(u)||, ||J(u)^T phi||] (J over the levels 1..N_t) with
both entries <= eps; the distance ||u^0 - u0|| = sqrt(h_x sum (u^0 - u0)^2) is
reported beside it.  At the saddle point u^0 = u0, A(u) = 0 and phi = lambda = 0,
so the limit is the implicit scheme's solution, as with u^0 held fixed.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import pdhg as opdhg
from .problem import Problem, time_coeffs


@dataclass
class LagrangeResult:
    u: np.ndarray            # (N_t+1, ...) including the iterated u^0
    phi: np.ndarray          # (N_t, ...)
    lam: np.ndarray          # (...): the multiplier of u^0 = u0
    iters: int
    res_primal: float
    res_dual: float
    init_dist: float         # ||u^0 - u0||
    converged: bool
    history: list = field(default_factory=list)   # [(n, Rp, Rd, ||u^0 - u0||)]


def lagrangian(prob: Problem, u: np.ndarray, phi: np.ndarray, lam: np.ndarray, u0: np.ndarray) -> float:
    """L(u, phi, lambda) as printed in Section 3.3 (u^0 = u[0] free)."""
    residual, _, _ = opdhg._ops(prob)
    a = residual(prob, u)
    return float(prob.ht * prob.hx * np.sum(phi * a) + prob.hx * np.sum(lam * (u[0] - u0)))


def j0t(prob: Problem, phi: np.ndarray) -> np.ndarray:
    """h_t J_0^T phi with J_0 = dA/du^0: the u^0 coefficients of the time differences of rows 0 and 1."""
    out = time_coeffs(prob.time, 0)[1] * phi[0]
    if prob.nt >= 2:
        out = out + time_coeffs(prob.time, 1)[2] * phi[1]
    return out


def init_dist(prob: Problem, u: np.ndarray, u0: np.ndarray) -> float:
    return float(np.sqrt(prob.hx * np.sum((u[0] - u0) ** 2)))


def run(prob: Problem, u0: np.ndarray, tau_u: float, tau_phi: float, tau_lam: float, eps: float = 0.0,
        max_iter: int = 1000, tau_u0: float = None, record: bool = False) -> LagrangeResult:
    """Algorithm 1 in the multiplier form from the initial guess u^l = u0 (all l, u^0 included),
    phi = 0, lambda = 0; stops at the first n with max(Rp, Rd) <= eps (eps = 0: exactly max_iter)."""
    residual, _, wnorm = opdhg._ops(prob)
    tau_u0 = 0.5 * tau_u if tau_u0 is None else tau_u0
    u0 = np.asarray(u0, dtype=np.float64)
    u = np.broadcast_to(u0, (prob.nt + 1,) + u0.shape).copy()
    phi = np.zeros((prob.nt,) + u0.shape)
    phibar = phi.copy()
    lam = np.zeros(u0.shape)
    lambar = lam.copy()
    hist = []
    rp = rd = float("inf")
    n = 0
    jt = opdhg.jt_operator(prob, u)
    for n in range(1, max_iter + 1):
        g0 = j0t(prob, phibar) + lambar          # uses the pre-update phibar, lambdabar
        u[1:] -= tau_u * jt(phibar)
        u[0] -= tau_u0 * g0
        r = residual(prob, u)
        s = opdhg.kd_solve_any(prob, r)
        phibar = phi + 2.0 * tau_phi * s
        phi = phi + tau_phi * s
        dl = tau_lam * (u[0] - u0)
        lambar = lam + 2.0 * dl
        lam = lam + dl
        jt = opdhg.jt_operator(prob, u)
        rp = wnorm(prob, r)
        rd = wnorm(prob, jt(phi))
        if record:
            hist.append((n, rp, rd, init_dist(prob, u, u0)))
        if not (np.isfinite(rp) and np.isfinite(rd)):
            break
        if max(rp, rd) <= eps:
            return LagrangeResult(u, phi, lam, n, rp, rd, init_dist(prob, u, u0), True, hist)
    return LagrangeResult(u, phi, lam, n, rp, rd, init_dist(prob, u, u0), False, hist)
