"""MI355X (gfx950) direct FFT pressure solve (N. Brown, "A comparison of
techniques for solving the Poisson equation in CFD", Section 2.1), with the
paper's matrix-free conjugate-gradient alternative (Section 2.2) on the same
operator.

The solvers run in the HIP library libpressure_solve.so behind the C ABI of
include/pressure_solve.h; this package is its thin Python binding
(``Plan``, ``BatchPlan``, ``CGSolver``, ``poisson_solve``) plus the seeded
synthetic workloads.
"""
from .binding import (BatchPlan, CGSolver, Plan, PressureSolveError, poisson_solve,  # noqa: F401
                      PRECISIONS)

__all__ = ["BatchPlan", "CGSolver", "Plan", "PressureSolveError", "poisson_solve", "PRECISIONS"]
