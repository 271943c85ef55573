"""Per-wavenumber identities that let a full-size solve be checked on a few
sampled horizontal wavenumbers, one oracle column solve each.

For a horizontal wavenumber (kx, ky) other than (0, 0) the solve decouples
into one vertical system per column (Section 2.1's method: horizontal
transform, tridiagonal solve per wavenumber, inverse transform), and the
mean-removal and gauge of the bordered system touch only the (0, 0) mode.
With s = 4 sin^2(pi kx/nx)/dx^2 + 4 sin^2(pi ky/ny)/dy^2 and the vertical
operator V = D^-1 T (T symmetric tridiagonal, D_k = rho_k dz_k):
  forward:  S b   at (kx, ky) = (-s I + V)^-1 b_hat
  adjoint:  S^T w at (kx, ky) = D (-s I + V)^-1 (D^-1 w_hat),
the latter because (-s I + V)^T = T D^-1 - s I = D (-s I + V) D^-1.
Both are checked against the oracle's full solves on the CPU
(tests/test_sampling_identities.py).
"""
import numpy as np

import oracle


def dft_at(x, kx, ky):
    """2D DFT coefficient (kx, ky) of every level, by a plain sum."""
    nz, ny, nx = x.shape
    ex = np.exp(-2j * np.pi * kx * np.arange(nx) / nx)
    ey = np.exp(-2j * np.pi * ky * np.arange(ny) / ny)
    return (x @ ex) @ ey


def horizontal_eigenvalue(kx, ky, nx, ny, dx, dy):
    return (4 * np.sin(np.pi * kx / nx) ** 2 / dx ** 2
            + 4 * np.sin(np.pi * ky / ny) ** 2 / dy ** 2)


def forward_column(b, kx, ky, dx, dy, dz, rho):
    """Coefficient (kx, ky) of S b, from the oracle's column solve."""
    nz, ny, nx = b.shape
    s = horizontal_eigenvalue(kx, ky, nx, ny, dx, dy)
    return oracle.column_solve(s, dft_at(b, kx, ky), dz, rho)


def adjoint_column(w, kx, ky, dx, dy, dz, rho):
    """Coefficient (kx, ky) of S^T w, from the oracle's column solve."""
    nz, ny, nx = w.shape
    s = horizontal_eigenvalue(kx, ky, nx, ny, dx, dy)
    D = np.asarray(rho) * np.asarray(dz)
    return D * oracle.column_solve(s, dft_at(w, kx, ky) / D, dz, rho)
