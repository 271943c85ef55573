"""Host-side parts of bench.py (no GPU): the fast CPU reference solve it
times next to the oracle reaches the oracle's result, and the benchmark
refuses more than one GPU."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2010_14132_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("shape,stretch,seed", [((5, 6, 8), 1.03, 1), ((10, 12, 16), 1.05, 2),
                                                ((1, 8, 8), 1.0, 3), ((7, 9, 18), 1.02, 4)])
def test_fast_cpu_reference_matches_oracle(shape, stretch, seed):
    nz, ny, nx = shape
    g = wl.stretched_grid(nx, ny, nz, stretch=stretch)
    g.dy = 37.0
    b = np.random.default_rng(seed).standard_normal(shape) + 0.4  # incompatible
    want = oracle.solve(b, g.dx, g.dy, g.dz, g.rho)
    got = bench.fast_cpu_solve(b, g.dx, g.dy, g.dz, g.rho, workers=2)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
