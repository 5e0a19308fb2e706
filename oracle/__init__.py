"""FP64 CPU oracle for the space-time primal-dual solver.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously
correct reference that the GPU path is checked against.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it;
the product library never calls it and shares no code with it.

Contents (each function cites the passage of Liu, Osher, Li and Shu, "A
primal-dual approach for solving conservation laws with implicit in time
approximations", that it follows):

* ``problem``   -- the problem description (flux, scheme, grid, constants).
* ``fd``        -- finite-difference residual A(u), Jacobian J(u), J(u)^T
                   (Sections 3.1-3.2).
* ``dg``        -- DG discretisations: the paper's P1 nodal upwind matrices
                   (Section 3.2.2, Appendix A) and a P2 Legendre local
                   Lax-Friedrichs scheme.
* ``precond``   -- the preconditioner K_d and its inverse (Section 2.2,
                   Section 3.3).
* ``pdhg``      -- Algorithm 1 with the initial level held fixed.
* ``newton``    -- a sequential Newton time march of the same implicit scheme
                   (defines the discrete solution independently of PDHG).
* ``adjoint``   -- gradient of a terminal loss with respect to u0 through the
                   implicit scheme (plain sparse solve of J^T mu = g).
* ``closed_form`` -- closed forms for linear upwind backward Euler.

Parity pins: see the oracle test files under ``tests/``.  Every function
here is pinned by at least one test against something other than itself
(a printed value of the paper, a closed form, brute force, or an
invariant) unless its docstring says "parity unpinned".
"""
from .problem import Problem  # noqa: F401
