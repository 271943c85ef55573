"""Batched solves in the withdrawn mode PS_BATCH_PLANS: every problem's own
plan solve captured into ONE hipGraph, the plans' streams being four lanes
forked from the capture's origin.  Skipped: its first run ended in a host
segmentation fault during that capture and the mode was withdrawn
(ps_batch_set_mode refuses it); batched solves now run in the lanes mode
(tests/test_gpu_batch_lanes.py).  Each problem
runs the single-solve kernels with its planning defaults, so the result must
equal a standalone plan's solve bit for bit; small problems are also checked
against the FP64 oracle."""
import time

import numpy as np
import pytest

import oracle
from paper_2010_14132_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skip(reason="withdrawn mode: its first run ended in a host segmentation fault "
                            "during the single capture over forked plan streams"),
]


def announce(msg):
    print("\n[gpu] " + msg, flush=True)


def relmax(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


# (n = nx = ny, nz, stretching): uneven sizes, a 3 * 2^k length, a 2^a 3^b one
SMALL = [(64, 32, 1.0), (96, 48, 1.02), (128, 64, 1.04), (48, 16, 1.01), (192, 32, 1.03),
         (32, 8, 1.0)]


def single(g, rhs, precision):
    from paper_2010_14132_amd import Plan
    plan = Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.rho, precision=precision)
    out = plan.solve(rhs)
    torch.cuda.synchronize()
    plan.close()
    return out


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_small_uneven_batch(precision):
    from paper_2010_14132_amd import BatchPlan
    announce("plan-graph batch of %d uneven problems %s" % (len(SMALL), precision))
    probs = [wl.stretched_smooth(n, n, nz, seed=4000 + i, dtype="f32", stretch=s)
             for i, (n, nz, s) in enumerate(SMALL)]
    dt = torch.float64 if precision == "fp64" else torch.float32
    batch = BatchPlan([p.grid for p in probs], precision=precision)
    rhs = [torch.from_numpy(p.rhs_exact()).to("cuda", dt) for p in probs]
    out = [torch.empty_like(r) for r in rhs]
    batch.solve(rhs, out)
    batch.status()
    first = [o.clone() for o in out]
    for rep in range(3):  # replays, with eager work between them
        for o in out:
            o.zero_()
        batch.solve(rhs, out)
        batch.status()
        for i, p in enumerate(probs):
            assert torch.equal(first[i], out[i]), (rep, i)
        torch.cuda.synchronize()
    tol = 1e-12 if precision == "fp64" else 1e-5
    for i, p in enumerate(probs):
        g = p.grid
        assert torch.equal(out[i], single(g, rhs[i], precision)), i
        ref = oracle.solve(p.rhs_exact(), g.dx, g.dy, g.dz, g.rho)
        got = out[i].double().cpu().numpy()
        assert relmax(got, ref) < tol, (i, relmax(got, ref))
    batch.close()


def test_plan_batch_recaptures_for_new_inputs_and_autotunes():
    from paper_2010_14132_amd import BatchPlan
    announce("plan-graph batch recapture + autotune")
    probs = [wl.stretched_smooth(n, n, nz, seed=4100 + i, dtype="f32", stretch=s)
             for i, (n, nz, s) in enumerate(SMALL[:3])]
    batch = BatchPlan([p.grid for p in probs], precision="fp32")
    rhs = [torch.from_numpy(p.rhs_as("f32")).cuda() for p in probs]
    out1 = [torch.empty_like(r) for r in rhs]
    out2 = [torch.empty_like(r) for r in rhs]
    batch.autotune(rhs, out1, reps=2)
    batch.solve(rhs, out1)
    batch.solve(rhs, out2)  # other output pointers: captured again
    rhs2 = [r.flip(1).contiguous() for r in rhs]
    out3 = [torch.empty_like(r) for r in rhs]
    batch.solve(rhs2, out3)  # other inputs too
    batch.status()
    for i, p in enumerate(probs):
        g = p.grid
        assert torch.equal(out1[i], out2[i])
        ref = oracle.solve(rhs2[i].double().cpu().numpy(), g.dx, g.dy, g.dz, g.rho)
        assert relmax(out3[i].double().cpu().numpy(), ref) < 1e-5
    batch.close()


def test_plan_batch_rejects_tile_modes():
    from paper_2010_14132_amd import BatchPlan
    from paper_2010_14132_amd.binding import PressureSolveError
    g = wl.stretched_smooth(32, 32, 8, seed=1, dtype="f32").grid
    batch = BatchPlan([g], precision="fp32", mode="phases")
    r = [torch.zeros((g.nz, g.ny, g.nx), device="cuda")]
    with pytest.raises(PressureSolveError):
        batch.solve(r, [torch.empty_like(r[0])])
    batch.close()
    with pytest.raises(PressureSolveError):
        BatchPlan([g], precision="fp32", mode="persistent")


def test_full_uneven_batch_48_plans():
    """The 48-problem recipe (nx = ny from {64..512} incl. 3*2^k sizes, nz
    from {32..128}, stretching in [1, 1.05], seed 4): every problem equal to
    its standalone FP32 plan, the two smallest against the oracle; replay
    time against the same solves issued one after another."""
    from paper_2010_14132_amd import BatchPlan, Plan
    probs = wl.batch_problems()
    npts = sum(p.grid.points for p in probs)
    announce("plan-graph batch of 48 uneven problems, %d points" % npts)
    batch = BatchPlan([p.grid for p in probs], precision="fp32")
    rhs = [torch.from_numpy(p.rhs_as("f32")).cuda() for p in probs]
    out = [torch.empty_like(r) for r in rhs]
    batch.solve(rhs, out)
    batch.status()
    plans = [Plan(p.grid.nx, p.grid.ny, p.grid.nz, p.grid.dx, p.grid.dy, p.grid.dz, p.grid.rho,
                  precision="fp32") for p in probs]
    seq = [torch.empty_like(r) for r in rhs]
    for pl, r, o in zip(plans, rhs, seq):
        pl.solve(r, out=o)
    torch.cuda.synchronize()
    for i in range(len(probs)):
        assert torch.equal(out[i], seq[i]), (i, probs[i].grid.nx, probs[i].grid.nz)
    small = sorted(range(len(probs)), key=lambda i: probs[i].grid.points)[:2]
    for i in small:
        g = probs[i].grid
        ref = oracle.solve(probs[i].rhs_exact(), g.dx, g.dy, g.dz, g.rho)
        assert relmax(out[i].double().cpu().numpy(), ref) < 1e-5

    def per_call(fn, n=20):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / n * 1e3

    def sequential():
        for pl, r, o in zip(plans, rhs, seq):
            pl.solve(r, out=o)

    t_graph = per_call(lambda: batch.solve(rhs, out))
    t_seq = per_call(sequential)
    print("48 problems: graph replay %.3f ms (%.0f Mpts/s), one stream eager %.3f ms"
          % (t_graph, npts / t_graph / 1e3, t_seq))
    for pl in plans:
        pl.close()
    batch.close()
