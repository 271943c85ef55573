"""Independent dense checker for the oracle (test code, not the oracle).

It writes the discrete operator down a second time, vectorised with numpy and
without any Fourier transform, assembles it as a dense matrix by applying it
to unit vectors, and solves the bordered system with LAPACK.  On tiny grids
this is brute force for the exact solution the oracle must reach.
"""
import numpy as np


def face_coefficients(dz, rho):
    """f_{k+1/2} for the nz-1 interior faces: mean face density over the
    centre-to-centre distance."""
    dz = np.asarray(dz)
    rho = np.asarray(rho)
    h = 0.5 * (dz[1:] + dz[:-1])
    return 0.5 * (rho[1:] + rho[:-1]) / h


def stencil(p, dx, dy, dz, rho):
    """A p for p of shape [nz][ny][nx] (complex rho allowed, for complex-step
    differentiation)."""
    p = np.asarray(p)
    lap = ((np.roll(p, -1, axis=2) - 2 * p + np.roll(p, 1, axis=2)) / dx ** 2
           + (np.roll(p, -1, axis=1) - 2 * p + np.roll(p, 1, axis=1)) / dy ** 2)
    fz = face_coefficients(dz, rho)                       # nz-1 faces
    flux = fz[:, None, None] * (p[1:] - p[:-1])           # upward flux through face k+1/2
    div = np.zeros(p.shape, dtype=np.result_type(p, fz))
    div[:-1] += flux
    div[1:] -= flux
    D = np.asarray(rho) * np.asarray(dz)
    return lap + div / D[:, None, None]


def dense_operator(shape, dx, dy, dz, rho):
    n = int(np.prod(shape))
    cols = []
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        cols.append(stencil(e.reshape(shape), dx, dy, dz, rho).ravel())
    return np.array(cols).T


def bordered(A):
    n = A.shape[0]
    K = np.zeros((n + 1, n + 1), dtype=A.dtype)
    K[:n, :n] = A
    K[:n, n] = 1
    K[n, :n] = 1
    return K


def dense_solve(b, dx, dy, dz, rho):
    A = dense_operator(b.shape, dx, dy, dz, rho)
    sol = np.linalg.solve(bordered(A), np.append(b.ravel(), 0.0))
    return sol[:-1].reshape(b.shape)


def dense_adjoint(w, dx, dy, dz, rho):
    A = dense_operator(w.shape, dx, dy, dz, rho)
    sol = np.linalg.solve(bordered(A).T, np.append(w.ravel(), 0.0))
    return sol[:-1].reshape(w.shape)
