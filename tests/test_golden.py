"""The stored fixture tests/golden/solve_8x6x5.txt (written by
tests/golden/make_golden.py, which calls only the oracle; the paper prints
no worked example).  CPU: the fixture matches its documented recipe, the
oracle still reproduces it, and the independent dense bordered solve agrees
with it.  GPU: the FP64 HIP solve through the C ABI reproduces it."""
import os

import numpy as np
import pytest

import oracle
from tests import dense_check as dc
from tests.golden import make_golden as mg

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "solve_8x6x5.txt")


def load():
    rows = {}
    with open(PATH) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, *vals = line.split()
            rows[key] = np.array([float(v) for v in vals])
    shape = (mg.NZ, mg.NY, mg.NX)
    return rows["dz"], rows["rho"], rows["b"].reshape(shape), rows["p"].reshape(shape)


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_fixture_matches_its_recipe():
    dz, rho, b, _ = load()
    rdz, rrho, rb = mg.recipe()
    assert np.array_equal(dz, rdz) and np.array_equal(rho, rrho) and np.array_equal(b, rb)


def test_oracle_reproduces_fixture():
    dz, rho, b, p = load()
    assert rel(oracle.solve(b, mg.DX, mg.DY, dz, rho), p) < 1e-14


def test_dense_bordered_solve_agrees_with_fixture():
    dz, rho, b, p = load()
    assert rel(dc.dense_solve(b, mg.DX, mg.DY, dz, rho), p) < 1e-12


@pytest.mark.gpu
def test_hip_fp64_solve_reproduces_fixture():
    torch = pytest.importorskip("torch")
    from paper_2010_14132_amd import Plan
    dz, rho, b, p = load()
    print("\n[gpu] golden 8x6x5 fp64", flush=True)
    plan = Plan(mg.NX, mg.NY, mg.NZ, mg.DX, mg.DY, dz, rho, precision="fp64")
    got = plan.solve(torch.from_numpy(b).cuda()).cpu().numpy()
    plan.close()
    assert rel(got, p) < 1e-12
