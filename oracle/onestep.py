"""One-time-step primal-dual solver (Algorithm 3, Section 3.5) -- oracle, test infrastructure only.

The implicit scheme is marched one step at a time.  Step l (l = 0..N_t-1)
is the initial-value problem on [l h_t, (l+1) h_t] discretised with one
implicit level: with u^l (and u^{l-1} for BDF2) known, the unknown
v = u^{l+1} solves

    A_l(v) = (c0 v + c1 u^l + c2 u^{l-1}) / h_t + F(v) = 0,

(c0, c1, c2) the coefficients of row l (BDF2 starts with backward Euler).
Algorithm 1 is applied to this N_x x 1 problem, started from v = u^l and
phi = phibar = 0, and stops when both residuals, measured in the L2 norm
over the time slice, sqrt(h_x sum z^2), are <= eps.

Readings (the paper states the algorithm only in words and pseudocode):

* The preconditioner of a step is the Gram reading of K_d with a single
  unknown level: B_t is the scalar c0/h_t, so
  K_l = (c0/h_t)^2 I + c^2 L_x + ghat^2 L_x^2, inverted by the FFT in x.
  For backward Euler this is K_d of the N_t = 1 space-time problem.  For DG
  P1 the same reading gives (c0/h_t)^2 I + c^2 G G^T on the two nodal planes,
  a 2x2 Hermitian matrix per Fourier mode over the cells.
* phi restarts from zero at every step (the paper sets only the initial
  guess of u).
* One pair of step sizes serves the whole march; the default is
  sqrt(0.95 / nu_max) with nu_max the largest eigenvalue of J^T K^{-1} J
  at u0 over the step operators the scheme uses (c0 = 1, and c0 = 3/2 for
  BDF2).  A step with c0 is the backward-Euler step of length h_t / c0.
* A step that reaches max_iter without meeting eps keeps its last iterate
  and the march goes on; a non-finite residual stops the march.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import fd
from . import pdhg as opdhg
from .precond import mode_shifts
from .problem import Problem, time_coeffs


@dataclass
class OneStepResult:
    u: np.ndarray                      # (N_t+1, N_x) or, DG P1, (N_t+1, 2, N_x); u[0] = u0
    phi: np.ndarray                    # (N_t, ...): the dual of step l at its n*
    step_iters: list                   # n*_l
    step_res: list                     # (Rp, Rd) of step l at n*_l
    converged: bool                    # every step met eps
    diverged: bool = False
    history: list = field(default_factory=list)


def slice_norm(prob: Problem, z: np.ndarray) -> float:
    """L2 norm over one time slice: sqrt(h_x sum_j z_j^2) (DG P1: the sum runs over both nodal planes,
    the nodal form of the space-time norm)."""
    return float(np.sqrt(prob.hx * np.sum(np.asarray(z) ** 2)))


def step_precond_symbol(prob: Problem, c0: float) -> np.ndarray:
    """Eigenvalues of K_l per FFT mode: (c0/h_t)^2 + c^2 mu_k + ghat^2 mu_k^2, or, for the full-symbol
    preconditioner, |c0/h_t + g_k|^2 (the one-level form of L_k L_k^*)."""
    if prob.precond_kind == "full":
        from .precond import full_symbol
        return np.abs(c0 / prob.ht + full_symbol(prob)) ** 2
    return (c0 / prob.ht) ** 2 + mode_shifts(prob)


def dg1_step_precond(prob: Problem, c0: float) -> np.ndarray:
    """DG P1: K_l per Fourier mode m over the cells, (c0/h_t)^2 I + c^2 G(theta_m) G(theta_m)^*, the
    one-level form of the DG preconditioner (G the unit-speed upwind P1 operator).  (nx, 2, 2)."""
    from . import dg1
    blocks = dg1.unit_upwind_blocks(prob)
    out = np.empty((prob.nx, 2, 2), dtype=np.complex128)
    for m in range(prob.nx):
        g = dg1.symbol(prob, 2.0 * np.pi * m / prob.nx, blocks)
        out[m] = (c0 / prob.ht) ** 2 * np.eye(2) + prob.precond_c ** 2 * (g @ g.conj().T)
    return out


def _step_operators(prob: Problem, c0: float):
    """(F, J_F^T apply, K_l^{-1}) of the one-level problem: finite differences on (nx,), DG P1 on the
    two nodal planes (2, nx)."""
    if prob.space == "dg_p1_upwind":
        from . import dg1
        kl = dg1_step_precond(prob, c0)

        def kinv(r):
            R = np.fft.fft(r, axis=-1)
            S = np.linalg.solve(kl, R.T[:, :, None])[:, :, 0].T
            return np.fft.ifft(S, axis=-1).real

        def jft(vv, psi):
            return (dg1.spatial_jacobian(prob, vv).T @ psi.ravel()).reshape(psi.shape)

        return (lambda vv: dg1.spatial_operator(prob, vv)), jft, kinv
    if prob.space == "dg_p2_llf":
        raise ValueError("the one-step oracle covers finite differences and DG P1")
    sym = step_precond_symbol(prob, c0)
    return ((lambda vv: fd.flux_operator(prob, vv)), (lambda vv, psi: fd.flux_jacobian(prob, vv).T @ psi),
            (lambda r: np.fft.ifft(np.fft.fft(r) / sym).real))


def solve_step(prob: Problem, row: int, u_prev: np.ndarray, u_prev2, tau_u: float, tau_phi: float,
               eps: float, max_iter: int, v_init=None, hist=None):
    """Algorithm 1 on the one-level problem of step `row`, started from v = u_prev (or v_init);
    returns (v, phi, n*, Rp, Rd).  hist: optional list that receives (n, Rp, Rd) per iteration."""
    c0, c1, c2 = time_coeffs(prob.time, row)
    known = c1 * u_prev + (c2 * u_prev2 if c2 != 0.0 else 0.0)
    ht = prob.ht
    flux, jft, kinv = _step_operators(prob, c0)
    v = np.array(u_prev if v_init is None else v_init, dtype=np.float64)
    phi = np.zeros_like(v)
    phibar = np.zeros_like(v)

    def jt(vv, psi):
        # J_l(v)^T psi with J_l(v) = (c0/h_t) I + dF(v)
        return c0 / ht * psi + jft(vv, psi)

    rp = rd = float("inf")
    n = 0
    for n in range(1, max_iter + 1):
        v = v - tau_u * jt(v, phibar)
        r = (c0 * v + known) / ht + flux(v)
        s = kinv(r)
        phibar = phi + 2.0 * tau_phi * s
        phi = phi + tau_phi * s
        rp = slice_norm(prob, r)
        rd = slice_norm(prob, jt(v, phi))
        if hist is not None:
            hist.append((n, rp, rd))
        if not (np.isfinite(rp) and np.isfinite(rd)):
            break
        if max(rp, rd) <= eps:
            break
    return v, phi, n, rp, rd


def auto_steps(prob: Problem, u0: np.ndarray, safety: float = 0.95, iters: int = 200):
    """sigma = tau = sqrt(safety / nu_max) over the step operators at u0.

    The step with coefficient c0 is the backward-Euler N_t = 1 problem with
    time step h_t / c0, whose nu_max Algorithm 1's power iteration gives."""
    c0s = [1.0] + ([1.5] if prob.time == "bdf2" and prob.nt > 1 else [])
    nm = 0.0
    for c0 in c0s:
        q = prob.with_(nt=1, time="be", t_final=prob.ht / c0)
        u = np.stack([u0, u0])
        nm = max(nm, opdhg.nu_max(q, u, iters))
    t = float(np.sqrt(safety / nm))
    return t, t, nm


def run(prob: Problem, u0: np.ndarray, eps: float, max_iter: int = 10000, tau_u: float = None,
        tau_phi: float = None) -> OneStepResult:
    """Algorithm 3 over l = 0..N_t-1."""
    if prob.space == "dg_p2_llf":
        raise ValueError("the one-step oracle covers finite differences and DG P1")
    if tau_u is None or tau_phi is None:
        tu, tp, _ = auto_steps(prob, u0)
        tau_u = tu if tau_u is None else tau_u
        tau_phi = tp if tau_phi is None else tau_phi
    u0 = np.asarray(u0, dtype=np.float64)
    u = np.empty((prob.nt + 1,) + u0.shape)
    u[0] = u0
    phi = np.zeros((prob.nt,) + u0.shape)
    its, res = [], []
    ok = True
    for l in range(prob.nt):
        v, ph, n, rp, rd = solve_step(prob, l, u[l], u[l - 1] if l >= 1 else None, tau_u, tau_phi, eps, max_iter)
        u[l + 1] = v
        phi[l] = ph
        its.append(n)
        res.append((rp, rd))
        if not (np.isfinite(rp) and np.isfinite(rd)):
            return OneStepResult(u, phi, its, res, False, True)
        ok = ok and max(rp, rd) <= eps
    return OneStepResult(u, phi, its, res, ok)
