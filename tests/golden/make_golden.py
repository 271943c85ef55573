"""Writes tests/golden/solve_8x6x5.txt: an FP64 oracle solve on a tiny
stretched grid, kept as a fixed regression value.

The paper prints no worked example (its only numbers, Table 1, need the
MONC test case), so this fixture is not a value from the paper: it is the
oracle's exact solution of the discrete bordered system (Section 2.1's
direct solve; readings R1-R6 of the discretisation) on the recipe below,
written by this script, which calls only oracle/.

Recipe: nz, ny, nx = 5, 6, 8; dx = 50, dy = 37 (m); dz_k = 20 * 1.1**k;
rho_k = exp(-z_k / 8000) at the cell centres z_k; b ~ N(0, 1) + 0.3
(incompatible on purpose) from numpy.random.default_rng(2024).

Run from the repository root:  python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

NZ, NY, NX = 5, 6, 8
DX, DY = 50.0, 37.0
SEED = 2024
PATH = os.path.join(HERE, "solve_8x6x5.txt")


def recipe():
    dz = 20.0 * 1.1 ** np.arange(NZ)
    zc = np.cumsum(dz) - 0.5 * dz
    rho = np.exp(-zc / 8000.0)
    b = np.random.default_rng(SEED).standard_normal((NZ, NY, NX)) + 0.3
    return dz, rho, b


def main():
    dz, rho, b = recipe()
    p = oracle.solve(b, DX, DY, dz, rho)
    with open(PATH, "w") as f:
        f.write("# FP64 oracle solve, shape nz ny nx = %d %d %d, dx %r dy %r, seed %d\n"
                % (NZ, NY, NX, DX, DY, SEED))
        f.write("# written by tests/golden/make_golden.py (oracle only); recipe in its docstring\n")
        f.write("dz " + " ".join("%.17g" % v for v in dz) + "\n")
        f.write("rho " + " ".join("%.17g" % v for v in rho) + "\n")
        f.write("b " + " ".join("%.17g" % v for v in b.ravel()) + "\n")
        f.write("p " + " ".join("%.17g" % v for v in p.ravel()) + "\n")
    print("wrote", PATH)


if __name__ == "__main__":
    main()
