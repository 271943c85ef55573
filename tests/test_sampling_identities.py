"""The per-wavenumber identities the full-size GPU tests sample with
(tests/sampling.py), checked against the oracle's full forward and adjoint
solves at a small size (no GPU).  A wrong sign, a missing D scaling or a
transposed operand in either identity fails here before it can pass or fail
a GPU test for the wrong reason."""
import numpy as np
import pytest

import oracle
from tests import sampling

NZ, NY, NX = 10, 12, 16
DX, DY = 50.0, 37.0
MODES = [(1, 0), (0, 1), (1, 1), (3, 5), (8, 6), (5, 11), (8, 0), (2, 7)]


def grid(seed):
    r = np.random.default_rng(seed)
    dz = 20.0 * 1.03 ** np.arange(NZ) * r.uniform(0.7, 1.3, NZ)
    rho = np.exp(-np.cumsum(dz) / 8000.0) * r.uniform(0.8, 1.2, NZ)
    return dz, rho


@pytest.mark.parametrize("kx,ky", MODES)
def test_forward_column_identity(kx, ky):
    dz, rho = grid(3)
    b = np.random.default_rng(4).standard_normal((NZ, NY, NX)) + 0.3
    p = oracle.solve(b, DX, DY, dz, rho)
    want = sampling.dft_at(p, kx, ky)
    got = sampling.forward_column(b, kx, ky, DX, DY, dz, rho)
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("kx,ky", MODES)
def test_adjoint_column_identity(kx, ky):
    dz, rho = grid(5)
    w = np.random.default_rng(6).standard_normal((NZ, NY, NX)) + 0.2
    lam = oracle.solve_adjoint(w, DX, DY, dz, rho)
    want = sampling.dft_at(lam, kx, ky)
    got = sampling.adjoint_column(w, kx, ky, DX, DY, dz, rho)
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


def test_adjoint_column_differs_from_forward():
    """With non-constant D the two identities give different columns, so the
    adjoint check cannot pass on a forward solve."""
    dz, rho = grid(5)
    w = np.random.default_rng(6).standard_normal((NZ, NY, NX))
    a = sampling.adjoint_column(w, 1, 1, DX, DY, dz, rho)
    f = sampling.forward_column(w, 1, 1, DX, DY, dz, rho)
    assert np.abs(a - f).max() > 1e-3 * np.abs(f).max()
