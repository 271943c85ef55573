"""Batched solves in the withdrawn tile-based mode (one kernel per phase over
the tiles of every problem), against the FP64 oracle and against the
single-problem plans.  Skipped: that mode shared its tile work list with the
persistent launch that did not complete on the GPU, and both were withdrawn
from the library (ps_batch_set_mode refuses them); batched solves now run in
the lanes mode (tests/test_gpu_batch_lanes.py)."""
import numpy as np
import pytest

import oracle
from paper_2010_14132_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skip(reason="withdrawn mode: the persistent launch did not complete on the GPU "
                            "and its cause was not found; the per-phase form shared its work "
                            "list and was withdrawn with it"),
]


def announce(msg):
    print("\n[gpu] " + msg, flush=True)


def relmax(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


SMALL = [(64, 32, 1.0), (96, 48, 1.02), (128, 64, 1.04), (48, 16, 1.01), (192, 32, 1.03),
         (32, 8, 1.0)]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_small_uneven_batch_vs_oracle(precision):
    from paper_2010_14132_amd import BatchPlan
    announce("batch of %d uneven problems %s" % (len(SMALL), precision))
    probs = [wl.stretched_smooth(n, n, nz, seed=4000 + i, dtype="f32", stretch=s)
             for i, (n, nz, s) in enumerate(SMALL)]
    dt = torch.float64 if precision == "fp64" else torch.float32
    batch = BatchPlan([p.grid for p in probs], precision=precision, mode="phases")
    rhs = [torch.from_numpy(p.rhs_exact()).to("cuda", dt) for p in probs]
    out = [torch.empty_like(r) for r in rhs]
    batch.solve(rhs, out)
    batch.status()
    torch.cuda.synchronize()
    first = [o.clone() for o in out]
    batch.solve(rhs, out)  # replay
    torch.cuda.synchronize()
    tol = 1e-12 if precision == "fp64" else 1e-5
    for i, p in enumerate(probs):
        g = p.grid
        ref = oracle.solve(p.rhs_exact(), g.dx, g.dy, g.dz, g.rho)
        got = out[i].double().cpu().numpy()
        assert relmax(got, ref) < tol, (i, relmax(got, ref))
        assert torch.equal(first[i], out[i])  # replay is deterministic
    info = batch.info()
    assert info["count"] == len(SMALL) and info["tiles"] > 0 and info["grid"] > 0


def test_batch_recaptures_for_new_pointers_and_autotunes():
    from paper_2010_14132_amd import BatchPlan
    announce("batch recapture + autotune")
    probs = [wl.stretched_smooth(n, n, nz, seed=4100 + i, dtype="f32", stretch=s)
             for i, (n, nz, s) in enumerate(SMALL[:3])]
    batch = BatchPlan([p.grid for p in probs], precision="fp32", mode="phases")
    rhs = [torch.from_numpy(p.rhs_as("f32")).cuda() for p in probs]
    out1 = [torch.empty_like(r) for r in rhs]
    out2 = [torch.empty_like(r) for r in rhs]
    batch.autotune(rhs, out1, reps=2)
    batch.solve(rhs, out1)
    batch.solve(rhs, out2)  # different pointers: captured again
    torch.cuda.synchronize()
    for a, b in zip(out1, out2):
        assert torch.equal(a, b)


def test_full_uneven_batch_48_vs_single_plans():
    """The 48-problem recipe (nx = ny from {64..512} incl. 3*2^k sizes, nz
    from {32..128}, stretching in [1, 1.05], seed 4) against the standalone
    FP32 plan of every problem, and two problems against the oracle."""
    from paper_2010_14132_amd import BatchPlan, Plan
    probs = wl.batch_problems()
    announce("batch of 48 uneven problems, %d points" % sum(p.grid.points for p in probs))
    batch = BatchPlan([p.grid for p in probs], precision="fp32", mode="phases")
    rhs = [torch.from_numpy(p.rhs_as("f32")).cuda() for p in probs]
    out = [torch.empty_like(r) for r in rhs]
    batch.solve(rhs, out)
    batch.status()
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        g = p.grid
        plan = Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.rho, precision="fp32")
        single = plan.solve(rhs[i])
        torch.cuda.synchronize()
        err = (out[i] - single).abs().max().item() / single.abs().max().item()
        assert err < 2e-5, (i, g.nx, g.nz, err)
        plan.close()
    small = sorted(range(len(probs)), key=lambda i: probs[i].grid.points)[:2]
    for i in small:
        g = probs[i].grid
        ref = oracle.solve(probs[i].rhs_exact(), g.dx, g.dy, g.dz, g.rho)
        assert relmax(out[i].double().cpu().numpy(), ref) < 1e-5
