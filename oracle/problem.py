"""Problem description used by the oracle (test infrastructure only).

The initial-value problem is the periodic scalar conservation law of
Section 2.1:  u_t + f(u)_x - (gamma(x) u_x)_x = 0,  u(x,0) = u0(x),
on [0, length) x [0, t_final].  The flux is the quadratic family of
Section 3.2.3, f(u) = alpha u^2 + beta u; the linear transport case of
Section 2.1 is alpha = 0, beta = a.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Callable, Optional

import numpy as np


@dataclass(frozen=True)
class Problem:
    nx: int
    nt: int
    length: float = 1.0
    t_final: float = 1.0
    # flux f(u) = alpha*u^2 + beta*u
    alpha: float = 0.0
    beta: float = 1.0
    gamma: float = 0.0                 # constant viscosity (centred diffusion)
    time: str = "be"                   # "be" | "bdf2"
    space: str = "fd_upwind"           # "fd_upwind" | "fd_lf" | "heat_var" | "dg_p2_llf" | "dg_p1_upwind"
    lf_speed: float = 0.0              # global Lax-Friedrichs constant (fd_lf)
    precond_c: float = 0.0             # c in K = -d_tt - c^2 d_xx + ghat^2 d_xxxx
    precond_gamma_hat: float = 0.0     # ghat
    precond_kind: str = "gram"         # "gram": K_d of Section 3.3 | "full": the Gram of the linearised operator
    gamma_fn: Optional[Callable] = field(default=None, compare=False)  # heat_var only

    @property
    def ht(self) -> float:
        """Uniform time step h_t = T / N_t (Section 3.1)."""
        return self.t_final / self.nt

    @property
    def hx(self) -> float:
        """Uniform mesh width h_x = b / N_x (Section 3.2)."""
        return self.length / self.nx

    @property
    def p(self) -> int:
        """Degrees of freedom per cell: 1 for finite differences, 3 for DG P2, 2 for DG P1."""
        return {"dg_p2_llf": 3, "dg_p1_upwind": 2}.get(self.space, 1)

    def f(self, u):
        return self.alpha * u * u + self.beta * u

    def fp(self, u):
        return 2.0 * self.alpha * u + self.beta

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)


def time_coeffs(time: str, row: int):
    """Coefficients (c0, c1, c2) of the time difference on row `row`.

    Row l of the implicit system reads (c0 u^{l+1} + c1 u^l + c2 u^{l-1})/h_t.
    Backward Euler (Section 3.1): (1, -1, 0).  BDF2 (end of Section 3.1):
    (3/2, -2, 1/2); the paper does not state the start-up step, and row 0
    uses backward Euler.
    """
    if time == "be" or row == 0:
        return 1.0, -1.0, 0.0
    if time == "bdf2":
        return 1.5, -2.0, 0.5
    raise ValueError(f"unknown time scheme {time!r}")


def default_constants(prob: Problem, u0: np.ndarray) -> Problem:
    """Fill the setup-time constants that default to data-dependent values.

    * Lax-Friedrichs constant: max |f'(u0)| when not given.
    * Preconditioner speed c: the paper takes c as an estimate of f'(u) from
      the initial data (Section 3.3); default max |f'(u0)|.
    """
    kw = {}
    if prob.space == "dg_p1_upwind":
        from .dg1 import default_speed
        if prob.precond_c <= 0.0:
            kw["precond_c"] = default_speed(prob, u0)
        return prob.with_(**kw) if kw else prob
    if prob.space == "dg_p2_llf":
        # DG: u0 is the (3, N_x) coefficient array; the speed is taken over the
        # cell-edge traces of u0_h (the states the local Lax-Friedrichs flux sees)
        from .dg import default_speed
        if prob.precond_c <= 0.0:
            kw["precond_c"] = default_speed(prob, u0)
        return prob.with_(**kw) if kw else prob
    if prob.space == "fd_lf" and prob.lf_speed <= 0.0:
        kw["lf_speed"] = float(np.max(np.abs(prob.fp(np.asarray(u0)))))
    if prob.precond_c <= 0.0 and prob.space != "heat_var":
        # the full-symbol preconditioner keeps the signed transport term: the mean speed of u0
        kw["precond_c"] = (float(np.mean(prob.fp(np.asarray(u0)))) if prob.precond_kind == "full"
                           else float(np.max(np.abs(prob.fp(np.asarray(u0))))))
    return prob.with_(**kw) if kw else prob
