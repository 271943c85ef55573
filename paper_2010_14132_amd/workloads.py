"""Seeded synthetic MONC-shaped workloads.

The paper drives its solvers with MONC's dry boundary-layer test case
(Section 3), which is not available here; these generators stand in for it.
They produce grids, density profiles and right-hand sides only: nothing in
this module performs any step of the pressure solve, so both the GPU path and
the CPU oracle can take their inputs from here.

All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64) in
FP64; FP32 workloads are the FP64 draws rounded once to FP32.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

DX = 50.0           # lateral spacing of every workload [m]
DZ_UNIFORM = 40.0   # level thickness of the uniform-grid workload [m]
DZ_BASE = 20.0      # lowest level thickness of the stretched grids [m]
STRETCH = 1.03      # geometric stretching factor of the stretched grids
SCALE_HEIGHT = 8000.0  # density scale height [m]


@dataclass
class Grid:
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: np.ndarray
    rho: np.ndarray

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def points(self) -> int:
        return self.nx * self.ny * self.nz


def uniform_grid(nx: int, ny: int, nz: int, dz: float = DZ_UNIFORM, dx: float = DX) -> Grid:
    """Uniform levels, constant density (the constant-coefficient case)."""
    return Grid(nx, ny, nz, dx, dx, np.full(nz, float(dz)), np.ones(nz))


def stretched_grid(nx: int, ny: int, nz: int, stretch: float = STRETCH,
                   dz0: float = DZ_BASE, dx: float = DX) -> Grid:
    """Levels dz_k = dz0 * stretch**k; density rho(z) = exp(-z / 8000 m) at
    the cell centres z_k = sum_{j<k} dz_j + dz_k / 2."""
    dz = dz0 * float(stretch) ** np.arange(nz, dtype=np.float64)
    zc = np.cumsum(dz) - 0.5 * dz
    rho = np.exp(-zc / SCALE_HEIGHT)
    return Grid(nx, ny, nz, dx, dx, dz, rho)


def white_field(rng: np.random.Generator, shape) -> np.ndarray:
    """I.i.d. N(0,1) with its global mean subtracted."""
    b = rng.standard_normal(shape)
    return b - b.mean()


def smooth_field(rng: np.random.Generator, grid: Grid, noise: float = 0.0) -> np.ndarray:
    """Gaussian field whose horizontal power spectrum falls as |k|^-2.

    Each level is an independent white N(0,1) draw whose 2D spectrum is
    multiplied by 1/|kappa| (kappa the physical wavenumber, the kappa = 0
    coefficient set to zero); the whole field is then scaled to unit variance.
    With ``noise`` > 0, noise * N(0,1) white noise drawn from the same
    generator is added.  Finally the global mean is subtracted.
    """
    nz, ny, nx = grid.shape
    kx = np.fft.rfftfreq(nx, d=grid.dx)
    ky = np.fft.fftfreq(ny, d=grid.dy)
    kap = 2 * np.pi * np.sqrt(kx[None, :] ** 2 + ky[:, None] ** 2)
    filt = np.zeros_like(kap)
    filt[kap > 0] = 1.0 / kap[kap > 0]
    out = np.empty(grid.shape)
    for k in range(nz):
        w = rng.standard_normal((ny, nx))
        out[k] = np.fft.irfft2(np.fft.rfft2(w) * filt, s=(ny, nx))
    out /= out.std()
    if noise:
        out += noise * rng.standard_normal(grid.shape)
    out -= out.mean()
    return out


@dataclass
class Problem:
    name: str
    grid: Grid
    rhs: np.ndarray           # FP64 draw
    dtype: str                # "f64" or "f32": the precision the solve runs in
    seed: int
    extra: dict = field(default_factory=dict)

    def rhs_as(self, dtype: str) -> np.ndarray:
        """Right-hand side rounded to the solve's precision."""
        return self.rhs.astype(np.float32 if dtype == "f32" else np.float64)

    def rhs_exact(self) -> np.ndarray:
        """The values the solve actually sees, promoted exactly to FP64 (the
        oracle's input for an FP32 solve)."""
        return self.rhs_as(self.dtype).astype(np.float64)


def uniform_white(seed: int = 0, nx: int = 32, ny: int = 32, nz: int = 16) -> Problem:
    """32^2 x 16, dz = 40 m, rho = 1, white RHS, FP64."""
    g = uniform_grid(nx, ny, nz)
    rng = np.random.default_rng(seed)
    return Problem("uniform_%dx%dx%d_white" % (nx, ny, nz), g, white_field(rng, g.shape), "f64", seed)


def stretched_smooth(nx: int, ny: int, nz: int, seed: int, dtype: str = "f64",
                     noise: float = 0.0, stretch: float = STRETCH) -> Problem:
    """Stretched levels, rho(z), smooth k^-2 RHS (+ optional white noise)."""
    g = stretched_grid(nx, ny, nz, stretch=stretch)
    rng = np.random.default_rng(seed)
    b = smooth_field(rng, g, noise=noise)
    return Problem("stretched_%dx%dx%d" % (nx, ny, nz), g, b, dtype, seed)


def plain_256() -> Problem:
    """256^2 x 64 stretched grid with rho(z), smooth RHS, FP64."""
    return stretched_smooth(256, 256, 64, seed=1, dtype="f64")


def precision_1024(dtype: str = "f32") -> Problem:
    """1024^2 x 128 stretched grid with rho(z), smooth RHS + 1 % white noise."""
    return stretched_smooth(1024, 1024, 128, seed=2, dtype=dtype, noise=0.01)


def differentiation_512() -> Problem:
    """512^2 x 128 stretched grid with rho(z), smooth RHS, FP32; also the
    loss weights w (seed 1003)."""
    p = stretched_smooth(512, 512, 128, seed=3, dtype="f32")
    p.extra["w"] = np.random.default_rng(1003).standard_normal(p.grid.shape)
    return p


BATCH_N = (64, 96, 128, 192, 256, 384, 512)
BATCH_NZ = (32, 48, 64, 96, 128)


def batch_sizes(count: int = 48, seed: int = 4):
    """Draw (n, nz, stretch) for each problem of the uneven batch."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice(BATCH_N))
        nz = int(rng.choice(BATCH_NZ))
        s = float(rng.uniform(1.0, 1.05))
        out.append((n, nz, s))
    return out


def batch_problems(count: int = 48, seed: int = 4, sizes=None):
    """Uneven batch: problem i is an n x n x nz stretched grid with its own
    stretching factor and its own smooth RHS (seed 4000 + i), FP32."""
    sizes = batch_sizes(count, seed) if sizes is None else sizes
    probs = []
    for i, (n, nz, s) in enumerate(sizes):
        probs.append(stretched_smooth(n, n, nz, seed=4000 + i, dtype="f32", stretch=s))
    return probs
