"""One pressure-projection step (ps_project): the divergence of a C-grid
velocity formed inside the forward x pass, the solve, and the pressure-
gradient correction; against the oracle's divergence, solve and gradient
(each pinned on the CPU), on the fast and the generic forward x kernels;
the corrected flow is divergence-free."""
import numpy as np
import pytest

import oracle
from paper_2010_14132_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5, "fp32_r2": 1e-5, "fp32_r1": 2e-7}


def announce(msg):
    print("\n[gpu] " + msg, flush=True)


def relmax(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def arch():
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


SHAPES = [(16, 32, 64), (5, 12, 18), (1, 8, 8), (9, 1, 16), (24, 48, 96), (7, 16, 1024),
          (33, 64, 256)]
FP32_HARD = (7, 16, 1024)  # see test_projection_fp32_forms_hard_case


@pytest.mark.parametrize("xvar", [None, 0], ids=["planned", "generic"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("precision", ["fp64", "fp32_r1", "fp32", "fp32_r2"])
def test_projection_step(tmp_path, precision, shape, xvar):
    from paper_2010_14132_amd import Plan
    from paper_2010_14132_amd.binding import PRECISIONS, tune_cache_load
    nz, ny, nx = shape
    if shape == FP32_HARD and precision in ("fp32", "fp32_r2"):
        pytest.skip("the unrefined FP32 forms on this case are bounded by FP32 transform "
                    "rounding (test_projection_fp32_forms_hard_case)")
    announce("projection %s %s x-variant %s" % (precision, shape, xvar))
    r = np.random.default_rng(nz * 7 + nx)
    g = wl.stretched_grid(nx, ny, nz, stretch=1.03)
    g.dz = g.dz * r.uniform(0.8, 1.2, nz)
    g.dy = 37.0
    dt = 2.5
    npdt = np.float64 if precision == "fp64" else np.float32
    u, v, w = (r.standard_normal(shape).astype(npdt) for _ in range(3))
    if xvar is not None:
        f = tmp_path / "tune.txt"
        f.write_text("%s %d %d %d %d %d 1 3 1 1 %d\n"
                     % (arch(), nx, ny, nz, PRECISIONS[precision], xvar, xvar))
        tune_cache_load(str(f))
    plan = Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.rho, precision=precision)
    if xvar is not None:
        plan.autotune()
        assert plan.info()["fft_variant_x"] == xvar
    ut, vt, wt = (torch.from_numpy(a).cuda() for a in (u, v, w))
    p = plan.project(ut, vt, wt, dt, correct=True)
    torch.cuda.synchronize()
    p = p.double().cpu().numpy()
    plan.close()
    b = oracle.divergence(u, v, w, g.dx, g.dy, g.dz, g.rho) / dt
    # the solve's input is the divergence rounded once to the plan's element
    # type (formed in FP64 inside the forward pass): as for every FP32 form,
    # the oracle solves that rounded input, promoted exactly
    if precision == "fp32_r1":
        # the refinement's residual uses the FP64 divergence itself
        pref = oracle.solve(b, g.dx, g.dy, g.dz, g.rho)
    else:
        pref = oracle.solve(b.astype(npdt).astype(np.float64), g.dx, g.dy, g.dz, g.rho)
    err = relmax(p, pref)
    gu, gv, gw = oracle.gradient(p, g.dx, g.dy, g.dz, g.rho)
    uc, vc, wc = (t.double().cpu().numpy() for t in (ut, vt, wt))
    tol_c = 1e-14 if precision == "fp64" else 1e-6
    scale = max(np.abs(u).max(), np.abs(v).max(), np.abs(w).max())
    for got, orig, gr in ((uc, u, gu), (vc, v, gv), (wc, w, gw)):
        assert np.abs(got - (orig - dt * gr)).max() < tol_c * scale
    assert np.array_equal(wc[0], w[0])  # the bottom boundary face is not touched
    div_after = oracle.divergence(uc, vc, wc, g.dx, g.dy, g.dz, g.rho)
    ratio = np.abs(div_after).max() / np.abs(b * dt).max()
    print("p rel_max %.3e, max|div| after / before %.3e" % (err, ratio))
    assert err < TOL[precision]
    assert ratio < (1e-9 if precision == "fp64" else 1e-4)


@pytest.mark.parametrize("precision", ["fp32", "fp32_r2"])
def test_projection_fp32_forms_hard_case(precision):
    """Without the physical-residual refinement the FP32 forms are bounded
    by FP32 transform rounding: the divergence of white noise is high-pass,
    its lowest modes (which dominate p) ~2 pi/1024 weaker than the typical
    mode on a 1024-wide grid, and the transforms' rounding costs them about
    1.4e-5 (the same figure as FP32 transforms emulated with scipy on the
    CPU, see the design notes).  Reported, bounded at 5e-5; the R1 form of
    test_projection_step meets 2e-7 on this case."""
    from paper_2010_14132_amd import Plan
    nz, ny, nx = 7, 16, 1024
    r = np.random.default_rng(nz * 7 + nx)
    g = wl.stretched_grid(nx, ny, nz, stretch=1.03)
    g.dz = g.dz * r.uniform(0.8, 1.2, nz)
    g.dy = 37.0
    u, v, w = (r.standard_normal((nz, ny, nx)).astype(np.float32) for _ in range(3))
    plan = Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.rho, precision=precision)
    p = plan.project(*(torch.from_numpy(a).cuda() for a in (u, v, w)), 2.5, correct=False)
    b = oracle.divergence(u, v, w, g.dx, g.dy, g.dz, g.rho) / 2.5
    pref = oracle.solve(b.astype(np.float32).astype(np.float64), g.dx, g.dy, g.dz, g.rho)
    err = relmax(p.double().cpu().numpy(), pref)
    print("%s 7x16x1024 white divergence: rel_max %.3e" % (precision, err))
    assert err < 5e-5
    plan.close()


def test_projection_refusals():
    from paper_2010_14132_amd import Plan
    from paper_2010_14132_amd.binding import PressureSolveError
    g = wl.stretched_grid(16, 16, 4)
    plan = Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.rho, precision="fp64")
    f = [torch.zeros((4, 16, 16), dtype=torch.float64, device="cuda") for _ in range(3)]
    with pytest.raises(PressureSolveError):
        plan.project(f[0], f[1], f[2], 0.0)
    with pytest.raises(PressureSolveError):
        plan.project(f[0], f[1], f[2], 1.0, out=f[0])
    plan.close()

