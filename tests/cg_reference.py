"""Plain numpy preconditioned conjugate gradients on M = -D A, the
symmetrised operator of the pressure solve (A applied by the oracle's
explicit stencil), as a reference for the HIP CG: the textbook PCG steps
in their usual order, FP64, no blocking or fusion.

The right-hand side is projected as in the direct solve (b' = b - mu, mu
the D-weighted mean) and scaled, rhs = -D b'; iterations stop when the
recurrence residual satisfies |r| <= rtol |rhs|; the result is shifted to
zero mean."""
import numpy as np

import oracle


def m_apply(x, dx, dy, dz, rho):
    D = np.asarray(rho) * np.asarray(dz)
    return -D[:, None, None] * oracle.apply(x, dx, dy, dz, rho)


def m_diagonal(shape, dx, dy, dz, rho):
    f, D = oracle.vertical_coefficients(dz, rho)
    d = D * (2 / dx ** 2 + 2 / dy ** 2) + f[:-1] + f[1:]
    return np.broadcast_to(d[:, None, None], shape)


def pcg(b, dx, dy, dz, rho, rtol, max_iter, precond="jacobi", x0=None):
    """(x, iterations, relative residual, residual history)."""
    nz, ny, nx = b.shape
    D = np.asarray(rho) * np.asarray(dz)
    mu = (D * b.sum(axis=(1, 2))).sum() / (D.sum() * nx * ny)
    rhs = -D[:, None, None] * (b - mu)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    dinv = 1.0 / m_diagonal(b.shape, dx, dy, dz, rho) if precond == "jacobi" else 1.0
    r = rhs - m_apply(x, dx, dy, dz, rho)
    z = r * dinv
    p = z.copy()
    rz = float((r * z).sum())
    rr = float((r * r).sum())
    rhs2 = float((rhs * rhs).sum())
    hist = [np.sqrt(rr / rhs2)]
    it = 0
    while rr > rtol * rtol * rhs2 and it < max_iter:
        q = m_apply(p, dx, dy, dz, rho)
        alpha = rz / float((p * q).sum())
        x += alpha * p
        r -= alpha * q
        z = r * dinv
        rz_new = float((r * z).sum())
        rr = float((r * r).sum())
        it += 1
        hist.append(np.sqrt(rr / rhs2))
        if rr <= rtol * rtol * rhs2:
            break
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x - x.mean(), it, np.sqrt(rr / rhs2), hist


def true_relative_residual(x, b, dx, dy, dz, rho):
    """|-D (b' - A x)| / |-D b'| with the oracle's stencil."""
    D = np.asarray(rho) * np.asarray(dz)
    nz, ny, nx = b.shape
    mu = (D * b.sum(axis=(1, 2))).sum() / (D.sum() * nx * ny)
    rhs = -D[:, None, None] * (b - mu)
    r = rhs - m_apply(x, dx, dy, dz, rho)
    return float(np.linalg.norm(r) / np.linalg.norm(rhs))
