"""Mesh refinement in time (Algorithm 2, Section 3.4) -- oracle, test infrastructure only.

Solve the initial-value problem on N x N_t0 with Algorithm 1, interpolate the
solution onto N x 2 N_t0 and use it as the initial guess there, doubling
until N_t is reached.  The paper only says "interpolate"; the reading used:

* u: linear interpolation in time.  Fine level 2l is coarse level l; fine
  level 2l+1 is the mean of coarse levels l and l+1 (level 0 stays u0).
* phi: one value per implicit row, i.e. per time interval.  Both fine rows
  2l and 2l+1 lie in coarse interval l and take its value (piecewise
  constant in time).

The coarse levels stop at their own tolerance or iteration cap; the finest
level is Algorithm 1 started from the interpolated pair (u, phi), with
phibar = phi.
"""
from __future__ import annotations

import numpy as np

from . import pdhg as opdhg
from .problem import Problem


def refine_in_time(u: np.ndarray, phi: np.ndarray):
    """(u, phi) on N_t levels -> (u, phi) on 2 N_t levels (shapes (N_t+1, ...), (N_t, ...))."""
    nt = u.shape[0] - 1
    uf = np.empty((2 * nt + 1,) + u.shape[1:])
    uf[0::2] = u
    uf[1::2] = 0.5 * (u[:-1] + u[1:])
    pf = np.empty((2 * nt,) + phi.shape[1:])
    pf[0::2] = phi
    pf[1::2] = phi
    return uf, pf


def levels(nt: int, nt_start: int):
    """Mesh sizes nt_start, 2 nt_start, ..., nt (nt / nt_start a power of two)."""
    out = [nt_start]
    while out[-1] < nt:
        out.append(2 * out[-1])
    if out[-1] != nt:
        raise ValueError("nt / nt_start must be a power of two")
    return out


def run(prob: Problem, u0: np.ndarray, nt_start: int, eps: float, max_iter: int = 100000,
        coarse_eps: float = None, coarse_max_iter: int = 100000, taus=None):
    """Algorithm 2.  taus: None (sqrt(0.95 / nu_max) per level by power iteration) or a
    callable nt -> tau.  Returns (final PdhgResult, [(nt, iterations) per level])."""
    ce = eps if coarse_eps is None else coarse_eps
    u = phi = None
    per_level = []
    nts = levels(prob.nt, nt_start)
    for k, nt in enumerate(nts):
        p = prob.with_(nt=nt)
        tau = taus(nt) if taus else opdhg.auto_steps(p, u0)[0]
        last = k == len(nts) - 1
        res = opdhg.run(p, u0, tau, tau, eps=eps if last else ce, max_iter=max_iter if last else coarse_max_iter,
                        u_init=u, phi_init=phi)
        per_level.append((nt, res.iters))
        if last:
            return res, per_level
        u, phi = refine_in_time(res.u, res.phi)
