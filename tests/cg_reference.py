"""Plain numpy Krylov references for the HIP solvers, FP64, the textbook
steps in their usual order, no blocking or fusion (A applied by the
oracle's explicit stencil).

pcg: preconditioned conjugate gradients on M = -D A, the symmetrised
operator of the pressure solve.  The right-hand side is projected as in the
direct solve (b' = b - mu, mu the D-weighted mean) and scaled,
rhs = -D b'; iterations stop when the recurrence residual satisfies
|r| <= rtol |rhs|; the result is shifted to zero mean.

bicgstab: van der Vorst's stabilised bi-conjugate gradients on A itself with
right preconditioning by K (the diagonal of A, or the identity): it solves
A K^-1 y = b' and x = K^-1 y, so the residual it tracks is b' - A x; it
stops when |r| <= rtol |b'|, after the half step or the full step; the
result is shifted to zero mean."""
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


def a_diagonal(dx, dy, dz, rho):
    """Diagonal of A per level."""
    f, D = oracle.vertical_coefficients(dz, rho)
    return -(2 / dx ** 2 + 2 / dy ** 2) - (f[:-1] + f[1:]) / D


def bicgstab(b, dx, dy, dz, rho, rtol, max_iter, precond="jacobi", x0=None):
    """(x, iterations, relative residual, residual history)."""
    nz, ny, nx = b.shape
    D = np.asarray(rho) * np.asarray(dz)
    mu = (D * b.sum(axis=(1, 2))).sum() / (D.sum() * nx * ny)
    rhs = b - mu
    kinv = 1.0 / a_diagonal(dx, dy, dz, rho) if precond == "jacobi" else np.ones(nz)
    kinv = kinv[:, None, None]
    x = np.zeros_like(b) if x0 is None else x0.copy()

    def a(v):
        return oracle.apply(v, dx, dy, dz, rho)

    r = rhs - a(x)
    rh = r.copy()
    rhs2 = float((rhs * rhs).sum())
    rr = float((r * r).sum())
    hist = [np.sqrt(rr / rhs2)]
    rho_old = alpha = omega = 1.0
    p = np.zeros_like(b)
    v = np.zeros_like(b)
    it = 0
    if rr <= rtol * rtol * rhs2:
        return x - x.mean(), 0, np.sqrt(rr / rhs2), hist
    while it < max_iter:
        rho_new = float((rh * r).sum())
        beta = 0.0 if it == 0 else (rho_new / rho_old) * (alpha / omega)
        p = r + beta * (p - omega * v)
        y = kinv * p
        v = a(y)
        alpha = rho_new / float((rh * v).sum())
        x = x + alpha * y
        s = r - alpha * v
        ss = float((s * s).sum())
        if ss <= rtol * rtol * rhs2:
            it += 1
            rr = ss
            hist.append(np.sqrt(rr / rhs2))
            break
        z = kinv * s
        t = a(z)
        omega = float((t * s).sum()) / float((t * t).sum())
        x = x + omega * z
        r = s - omega * t
        rr = float((r * r).sum())
        it += 1
        hist.append(np.sqrt(rr / rhs2))
        rho_old = rho_new
        if rr <= rtol * rtol * rhs2:
            break
    return x - x.mean(), it, np.sqrt(rr / rhs2), hist


def true_relative_residual_a(x, b, dx, dy, dz, rho):
    """|b' - A x| / |b'| with the oracle's stencil."""
    D = np.asarray(rho) * np.asarray(dz)
    nz, ny, nx = b.shape
    mu = (D * b.sum(axis=(1, 2))).sum() / (D.sum() * nx * ny)
    rhs = b - mu
    r = rhs - oracle.apply(x, dx, dy, dz, rho)
    return float(np.linalg.norm(r) / np.linalg.norm(rhs))
