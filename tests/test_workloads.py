"""The seeded input generators (CPU): the same seed gives identical bytes and
another seed different ones, and each recipe has the structure it states --
geometric level thicknesses and the exponential density at the cell
centres, a zero-mean unit-variance smooth field whose horizontal spectrum
falls as 1/|kappa| per level, the 48-problem batch drawn from its size sets,
and FP32 workloads that are the FP64 draws rounded once."""
import numpy as np
import pytest

from paper_2010_14132_amd import workloads as wl


def test_same_seed_same_bytes_other_seed_differs():
    a = wl.stretched_smooth(64, 48, 8, seed=5, noise=0.01)
    b = wl.stretched_smooth(64, 48, 8, seed=5, noise=0.01)
    c = wl.stretched_smooth(64, 48, 8, seed=6, noise=0.01)
    assert a.rhs.tobytes() == b.rhs.tobytes()
    assert a.grid.dz.tobytes() == b.grid.dz.tobytes() and a.grid.rho.tobytes() == b.grid.rho.tobytes()
    assert a.rhs.tobytes() != c.rhs.tobytes()
    assert wl.uniform_white(seed=3).rhs.tobytes() == wl.uniform_white(seed=3).rhs.tobytes()
    assert wl.batch_sizes() == wl.batch_sizes()


def test_stretched_grid_recipe():
    g = wl.stretched_grid(32, 16, 12, stretch=1.03)
    k = np.arange(12)
    assert np.allclose(g.dz, 20.0 * 1.03 ** k, rtol=1e-15, atol=0)
    zc = np.array([g.dz[:j].sum() + g.dz[j] / 2 for j in range(12)])
    assert np.allclose(g.rho, np.exp(-zc / 8000.0), rtol=1e-14, atol=0)
    assert g.dx == g.dy == 50.0 and g.shape == (12, 16, 32) and g.points == 12 * 16 * 32
    u = wl.uniform_grid(8, 8, 4)
    assert np.all(u.dz == 40.0) and np.all(u.rho == 1.0)


def test_smooth_field_spectrum_and_moments():
    g = wl.stretched_grid(64, 64, 6)
    f = wl.smooth_field(np.random.default_rng(11), g)
    assert abs(f.mean()) < 1e-12
    assert abs(f.std() - 1.0) < 1e-12  # the mean was zero before removal
    # per level, the zero wavenumber is absent and the power falls as 1/|k|^2:
    # the filtered spectrum times |kappa| is white, so its radial average is flat
    kx = np.fft.rfftfreq(64, d=g.dx)
    ky = np.fft.fftfreq(64, d=g.dy)
    kap = 2 * np.pi * np.sqrt(kx[None, :] ** 2 + ky[:, None] ** 2)
    spec = np.fft.rfft2(f, axes=(1, 2))
    white = np.abs(spec) ** 2 * kap ** 2
    lo = white[:, (kap > 0) & (kap < np.median(kap[kap > 0]))].mean()
    hi = white[:, kap >= np.median(kap[kap > 0])].mean()
    assert 0.7 < lo / hi < 1.4
    # the level means (kappa = 0) are only the global-mean removal's residue
    assert np.abs(spec[:, 0, 0]).max() < 1e-9 * np.abs(spec).max()


def test_batch_recipe():
    sizes = wl.batch_sizes()
    assert len(sizes) == 48
    for n, nz, s in sizes:
        assert n in wl.BATCH_N and nz in wl.BATCH_NZ and 1.0 <= s <= 1.05
    small = [(64, 32, 1.02), (96, 48, 1.0), (64, 8, 1.05)]  # the recipe on small sizes
    probs = wl.batch_problems(sizes=small)
    for i, p in enumerate(probs):
        n, nz, s = small[i]
        assert p.grid.shape == (nz, n, n) and p.dtype == "f32" and p.seed == 4000 + i
        assert np.allclose(p.grid.dz, 20.0 * s ** np.arange(nz), rtol=1e-14, atol=0)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_precision_rounding(dtype):
    p = wl.stretched_smooth(32, 16, 4, seed=2, dtype=dtype, noise=0.01)
    x = p.rhs_exact()
    assert x.dtype == np.float64
    if dtype == "f32":
        assert np.array_equal(x, p.rhs.astype(np.float32).astype(np.float64))
        assert not np.array_equal(x, p.rhs)
    else:
        assert np.array_equal(x, p.rhs)
