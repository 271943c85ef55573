"""MI355X (gfx950) direct FFT pressure solve (N. Brown, "A comparison of
techniques for solving the Poisson equation in CFD", Section 2.1).

The solve runs in the HIP library libpressure_solve.so behind the C ABI of
include/pressure_solve.h; this package is its thin Python binding
(``Plan``, ``poisson_solve``) plus the seeded synthetic workloads.
"""
from .binding import BatchPlan, Plan, PressureSolveError, poisson_solve, PRECISIONS  # noqa: F401

__all__ = ["BatchPlan", "Plan", "PressureSolveError", "poisson_solve", "PRECISIONS"]
