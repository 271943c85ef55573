"""The numpy CG reference (tests/cg_reference.py) pinned on the CPU: it
converges to the oracle's direct solve (the exact solution of the same
discrete system) on stretched grids with an incompatible right-hand side,
its true residual meets the tolerance, Jacobi preconditioning does not take
more iterations than none on a stretched grid, and a warm start from the
solution stops at once."""
import numpy as np
import pytest

import oracle
from paper_2010_14132_amd import workloads as wl
from tests import cg_reference as cg


def grid(nx, ny, nz, seed):
    r = np.random.default_rng(seed)
    g = wl.stretched_grid(nx, ny, nz, stretch=1.04)
    g.dz = g.dz * r.uniform(0.8, 1.2, nz)
    g.dy = 37.0
    return g


@pytest.mark.parametrize("shape,seed", [((6, 8, 10), 1), ((9, 12, 16), 2), ((1, 8, 8), 3),
                                        ((12, 1, 6), 4)])
@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_reference_cg_converges_to_the_direct_solve(shape, seed, precond):
    nz, ny, nx = shape
    g = grid(nx, ny, nz, seed)
    b = np.random.default_rng(seed + 10).standard_normal(shape) + 0.5
    want = oracle.solve(b, g.dx, g.dy, g.dz, g.rho)
    x, it, rel, hist = cg.pcg(b, g.dx, g.dy, g.dz, g.rho, 1e-13, 5000, precond)
    assert rel <= 1e-13 and it < 5000
    assert cg.true_relative_residual(x, b, g.dx, g.dy, g.dz, g.rho) < 1e-11
    assert np.abs(x - want).max() < 1e-8 * np.abs(want).max()


def test_jacobi_helps_and_warm_start_stops():
    g = grid(16, 16, 24, 5)
    b = np.random.default_rng(6).standard_normal((24, 16, 16))
    _, it_none, _, _ = cg.pcg(b, g.dx, g.dy, g.dz, g.rho, 1e-8, 5000, "none")
    _, it_jac, _, _ = cg.pcg(b, g.dx, g.dy, g.dz, g.rho, 1e-8, 5000, "jacobi")
    assert it_jac <= it_none
    exact = oracle.solve(b, g.dx, g.dy, g.dz, g.rho)
    _, it0, rel0, _ = cg.pcg(b, g.dx, g.dy, g.dz, g.rho, 1e-8, 5000, "jacobi", x0=exact)
    assert it0 == 0 and rel0 < 1e-8


@pytest.mark.parametrize("shape,seed", [((6, 8, 10), 1), ((9, 12, 16), 2), ((1, 8, 8), 3),
                                        ((12, 1, 6), 4)])
@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_reference_bicgstab_converges_to_the_direct_solve(shape, seed, precond):
    """The numpy BiCGStab reference on A itself (not symmetric on these
    stretched grids) reaches the oracle's exact solution of the bordered
    system, with its true residual within the tolerance."""
    nz, ny, nx = shape
    g = grid(nx, ny, nz, seed)
    b = np.random.default_rng(seed + 10).standard_normal(shape) + 0.5
    want = oracle.solve(b, g.dx, g.dy, g.dz, g.rho)
    x, it, rel, hist = cg.bicgstab(b, g.dx, g.dy, g.dz, g.rho, 1e-12, 5000, precond)
    assert rel <= 1e-12 and it < 5000
    assert cg.true_relative_residual_a(x, b, g.dx, g.dy, g.dz, g.rho) < 1e-10
    assert np.abs(x - want).max() < 1e-8 * np.abs(want).max()


def test_bicgstab_warm_start_and_nonsymmetric_operator():
    g = grid(16, 16, 24, 5)
    b = np.random.default_rng(6).standard_normal((24, 16, 16))
    exact = oracle.solve(b, g.dx, g.dy, g.dz, g.rho)
    _, it0, rel0, _ = cg.bicgstab(b, g.dx, g.dy, g.dz, g.rho, 1e-8, 5000, "jacobi", x0=exact)
    assert it0 == 0 and rel0 < 1e-8
    # A is not symmetric on a stretched grid (so BiCGStab, not CG, applies
    # to it directly) while -D A is
    rng = np.random.default_rng(7)
    u, w = rng.standard_normal((2, 24, 16, 16))
    au = oracle.apply(u, g.dx, g.dy, g.dz, g.rho)
    aw = oracle.apply(w, g.dx, g.dy, g.dz, g.rho)
    assert abs((w * au).sum() - (u * aw).sum()) > 1e-6 * np.abs(w * au).sum()
    mu = cg.m_apply(u, g.dx, g.dy, g.dz, g.rho)
    mw = cg.m_apply(w, g.dx, g.dy, g.dz, g.rho)
    assert abs((w * mu).sum() - (u * mw).sum()) < 1e-12 * np.abs(w * mu).sum()
