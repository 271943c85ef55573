"""FP64 CPU oracle for the direct FFT pressure solve -- test infrastructure.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library
(``paper_2010_14132_amd``) never imports, links or calls it, and the two share
no code: the oracle is plain C (``pressure_oracle.c``) compiled with gcc, the
product is HIP compiled with hipcc.

Every function takes and returns numpy arrays in the level-major layout
``[nz][ny][nx]`` (x fastest).  See ``pressure_oracle.c`` for the definitions
(paper Section 2.1: forward transform per level, one tridiagonal solve per
wavenumber column, backward transform).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pressure_oracle.c")
_LIB = os.path.join(_HERE, "libpressure_oracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)


_LIB_ASAN = os.path.join(_HERE, "libpressure_oracle_asan.so")


def build(force: bool = False, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math); with
    sanitize, a variant instrumented with AddressSanitizer and
    UndefinedBehaviorSanitizer (loaded when PS_ORACLE_SANITIZE is set, with
    gcc's ASan runtime preloaded)."""
    lib = _LIB_ASAN if sanitize else _LIB
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        tmp = lib + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        if sanitize:
            cmd[1:1] = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        "-fno-omit-frame-pointer", "-g"]
        subprocess.check_call(cmd)
        os.replace(tmp, lib)
    return lib


def _load():
    global _lib
    if _lib is None:
        sanitize = bool(os.environ.get("PS_ORACLE_SANITIZE"))
        lib = ctypes.CDLL(build(sanitize=sanitize))
        i, d = ctypes.c_int, ctypes.c_double
        grid = [i, i, i, d, d, _D, _D]
        lib.oracle_solve.argtypes = grid + [_D, _D]
        lib.oracle_solve_adjoint.argtypes = grid + [_D, _D]
        lib.oracle_apply.argtypes = grid + [_D, _D]
        lib.oracle_grad_rho.argtypes = grid + [_D, _D, _D]
        lib.oracle_dft2_forward.argtypes = [i, i, i, _D, _D]
        lib.oracle_dft2_inverse.argtypes = [i, i, i, _D, _D]
        lib.oracle_column_solve.argtypes = [i, _D, _D, d, _D, _D, _D, _D]
        lib.oracle_vertical_coefficients.argtypes = [i, _D, _D, _D, _D]
        lib.oracle_num_threads.argtypes = []
        lib.oracle_divergence.argtypes = grid + [_D, _D, _D, _D]
        lib.oracle_gradient.argtypes = grid + [_D, _D, _D, _D]
        for fn in (lib.oracle_solve, lib.oracle_solve_adjoint, lib.oracle_apply,
                   lib.oracle_grad_rho, lib.oracle_dft2_forward, lib.oracle_dft2_inverse,
                   lib.oracle_column_solve, lib.oracle_vertical_coefficients,
                   lib.oracle_num_threads, lib.oracle_divergence, lib.oracle_gradient):
            fn.restype = ctypes.c_int
        _lib = lib
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError("oracle %s failed with status %d" % (what, rc))


def _grid_args(dx, dy, dz, rho):
    dz = _f64(dz)
    rho = _f64(rho)
    return dz, rho


def solve(b, dx, dy, dz, rho) -> np.ndarray:
    """p = S b: the p-block of [[A,1],[1^T,0]] [p; mu] = [b; 0]."""
    b = _f64(b)
    nz, ny, nx = b.shape
    dz, rho = _grid_args(dx, dy, dz, rho)
    p = np.empty_like(b)
    _check(_load().oracle_solve(nx, ny, nz, float(dx), float(dy), _ptr(dz), _ptr(rho),
                                _ptr(b), _ptr(p)), "solve")
    return p


def solve_adjoint(w, dx, dy, dz, rho) -> np.ndarray:
    """lam = S^T w: the lambda-block of [[A^T,1],[1^T,0]] [lam; nu] = [w; 0]."""
    w = _f64(w)
    nz, ny, nx = w.shape
    dz, rho = _grid_args(dx, dy, dz, rho)
    lam = np.empty_like(w)
    _check(_load().oracle_solve_adjoint(nx, ny, nz, float(dx), float(dy), _ptr(dz),
                                        _ptr(rho), _ptr(w), _ptr(lam)), "solve_adjoint")
    return lam


def apply(p, dx, dy, dz, rho) -> np.ndarray:
    """A p by the explicit 7-point stencil."""
    p = _f64(p)
    nz, ny, nx = p.shape
    dz, rho = _grid_args(dx, dy, dz, rho)
    out = np.empty_like(p)
    _check(_load().oracle_apply(nx, ny, nz, float(dx), float(dy), _ptr(dz), _ptr(rho),
                                _ptr(p), _ptr(out)), "apply")
    return out


def grad_rho(lam, p, dx, dy, dz, rho) -> np.ndarray:
    """g_k = -lam^T (dA/drho_k) p for each level k."""
    lam = _f64(lam)
    p = _f64(p)
    nz, ny, nx = p.shape
    dz, rho = _grid_args(dx, dy, dz, rho)
    g = np.empty(nz)
    _check(_load().oracle_grad_rho(nx, ny, nz, float(dx), float(dy), _ptr(dz), _ptr(rho),
                                   _ptr(lam), _ptr(p), _ptr(g)), "grad_rho")
    return g


def dft2_forward(x) -> np.ndarray:
    """Unnormalised forward 2D DFT of every level; half spectrum
    complex array [nz][ny][nx//2+1]."""
    x = _f64(x)
    nz, ny, nx = x.shape
    out = np.empty((nz, ny, nx // 2 + 1, 2))
    _check(_load().oracle_dft2_forward(nx, ny, nz, _ptr(x), _ptr(out)), "dft2_forward")
    return out[..., 0] + 1j * out[..., 1]


def dft2_inverse(X, nx: int) -> np.ndarray:
    """Backward 2D DFT with 1/(nx*ny) of a half spectrum [nz][ny][nx//2+1]."""
    X = np.asarray(X)
    nz, ny, hx = X.shape
    assert hx == nx // 2 + 1
    buf = np.ascontiguousarray(np.stack([X.real, X.imag], axis=-1).astype(np.float64))
    out = np.empty((nz, ny, nx))
    _check(_load().oracle_dft2_inverse(nx, ny, nz, _ptr(buf), _ptr(out)), "dft2_inverse")
    return out


def column_solve(s, r, dz, rho) -> np.ndarray:
    """Solve (-s I + V) x = r on one column (complex r), s > 0."""
    r = np.asarray(r, dtype=np.complex128)
    nz = r.shape[0]
    dz = _f64(dz)
    rho = _f64(rho)
    rr, ri = _f64(r.real), _f64(r.imag)
    xr, xi = np.empty(nz), np.empty(nz)
    _check(_load().oracle_column_solve(nz, _ptr(dz), _ptr(rho), float(s), _ptr(rr), _ptr(ri),
                                       _ptr(xr), _ptr(xi)), "column_solve")
    return xr + 1j * xi


def vertical_coefficients(dz, rho):
    """(f, D): f[0]=f[nz]=0, f[k]=f_{k-1/2}; D[k]=rho_k dz_k."""
    dz = _f64(dz)
    rho = _f64(rho)
    nz = dz.shape[0]
    f = np.empty(nz + 1)
    D = np.empty(nz)
    _check(_load().oracle_vertical_coefficients(nz, _ptr(dz), _ptr(rho), _ptr(f), _ptr(D)),
           "vertical_coefficients")
    return f, D


def divergence(u, v, w, dx, dy, dz, rho) -> np.ndarray:
    """Anelastic divergence of C-grid velocities (see pressure_oracle.c)."""
    u, v, w = _f64(u), _f64(v), _f64(w)
    nz, ny, nx = u.shape
    dz, rho = _grid_args(dx, dy, dz, rho)
    out = np.empty_like(u)
    _check(_load().oracle_divergence(nx, ny, nz, float(dx), float(dy), _ptr(dz), _ptr(rho),
                                     _ptr(u), _ptr(v), _ptr(w), _ptr(out)), "divergence")
    return out


def gradient(p, dx, dy, dz, rho):
    """(gu, gv, gw): the pressure gradient on the u, v and w faces."""
    p = _f64(p)
    nz, ny, nx = p.shape
    dz, rho = _grid_args(dx, dy, dz, rho)
    gu, gv, gw = np.empty_like(p), np.empty_like(p), np.empty_like(p)
    _check(_load().oracle_gradient(nx, ny, nz, float(dx), float(dy), _ptr(dz), _ptr(rho),
                                   _ptr(p), _ptr(gu), _ptr(gv), _ptr(gw)), "gradient")
    return gu, gv, gw


def num_threads() -> int:
    return int(_load().oracle_num_threads())
