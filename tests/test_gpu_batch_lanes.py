"""Batched solves (mode PS_BATCH_LANES): problems of uneven sizes dealt to
lanes, each lane's solves captured into one hipGraph and the lane graphs
replayed side by side.  Every problem runs its own plan's kernels, so the
batched result must equal the standalone plan's solve bit for bit; the small
problems are also checked against the FP64 oracle, the large ones on sampled
wavenumber columns (one oracle column solve each)."""
import time

import numpy as np
import pytest

import oracle
from paper_2010_14132_amd import workloads as wl
from tests import sampling

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def announce(msg):
    print("\n[gpu] " + msg, flush=True)


def relmax(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


# (n = nx = ny, nz, stretching): uneven sizes, 3 * 2^k lengths, one level
SMALL = [(64, 32, 1.0), (96, 48, 1.02), (128, 64, 1.04), (48, 16, 1.01), (192, 32, 1.03),
         (32, 8, 1.0), (16, 1, 1.0)]

SAMPLE_MODES = [(1, 0), (0, 1), (1, 1), (3, 7), (5, 2)]


def standalone(grids, rhs, precision, autotune=False):
    from paper_2010_14132_amd import Plan
    outs = []
    for g, r in zip(grids, rhs):
        plan = Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.rho, precision=precision)
        if autotune:  # equal shapes: the tune cache gives the batch's choice
            plan.autotune(reps=2)
        outs.append(plan.solve(r))
        torch.cuda.synchronize()
        plan.close()
    return outs


def check_oracle(probs, out, tol):
    """Full oracle solve for problems up to 2^20 points, sampled wavenumber
    columns for larger ones."""
    for i, p in enumerate(probs):
        g = p.grid
        got = out[i].double().cpu().numpy()
        b = p.rhs_exact()
        if g.points <= 1 << 20:
            ref = oracle.solve(b, g.dx, g.dy, g.dz, g.rho)
            err = relmax(got, ref)
        else:
            scale, errs = 0.0, []
            for kx, ky in SAMPLE_MODES:
                want = sampling.forward_column(b, kx, ky, g.dx, g.dy, g.dz, g.rho)
                have = sampling.dft_at(got, kx, ky)
                scale = max(scale, np.abs(want).max())
                errs.append(np.abs(have - want).max())
            err = max(errs) / scale
        assert err < tol, (i, g.nx, g.nz, err)


@pytest.mark.parametrize("lanes,in_order", [(1, True), (3, True), (3, False)])
@pytest.mark.parametrize("precision", ["fp32", "fp64", "fp32_r2", "fp32_r1"])
def test_small_uneven_batch(precision, lanes, in_order):
    """Both FP64-column orders: in order on the lanes (the default) and each
    plan's own placement (forked onto its second stream inside the capture)."""
    from paper_2010_14132_amd import BatchPlan
    announce("batch of %d uneven problems %s, %d lanes, FP64 columns %s"
             % (len(SMALL), precision, lanes, "in order" if in_order else "forked"))
    probs = [wl.stretched_smooth(n, n, nz, seed=4000 + i, dtype="f32", stretch=s)
             for i, (n, nz, s) in enumerate(SMALL)]
    dt = torch.float64 if precision == "fp64" else torch.float32
    batch = BatchPlan([p.grid for p in probs], precision=precision, lanes=lanes)
    assert batch.info() == {"count": len(SMALL), "lanes": lanes, "fp64_in_order": True}
    batch.set_fp64_order(in_order)
    assert batch.info()["fp64_in_order"] == in_order
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
        for i in range(len(probs)):
            assert torch.equal(first[i], out[i]), (rep, i)
    single = standalone([p.grid for p in probs], rhs, precision)
    for i in range(len(probs)):
        assert torch.equal(out[i], single[i]), i
    tol = 1e-12 if precision == "fp64" else (2e-7 if precision == "fp32_r1" else 1e-5)
    check_oracle(probs, out, tol)
    batch.close()


def test_batch_recaptures_for_new_pointers_and_autotunes():
    from paper_2010_14132_amd import BatchPlan
    announce("batch recapture + autotune")
    probs = [wl.stretched_smooth(n, n, nz, seed=4100 + i, dtype="f32", stretch=s)
             for i, (n, nz, s) in enumerate(SMALL[:4])]
    batch = BatchPlan([p.grid for p in probs], precision="fp32")
    rhs = [torch.from_numpy(p.rhs_as("f32")).cuda() for p in probs]
    out1 = [torch.empty_like(r) for r in rhs]
    out2 = [torch.empty_like(r) for r in rhs]
    batch.autotune(rhs, out1, reps=2)
    assert batch.info()["lanes"] in (1, 2, 4)
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


def test_batch_follows_the_callers_stream():
    """Work queued on the caller's stream before the batched solve (writing
    the right-hand sides) is complete when the lanes start, and work queued
    after it sees the results."""
    from paper_2010_14132_amd import BatchPlan
    announce("batch ordering on a caller stream")
    probs = [wl.stretched_smooth(n, n, nz, seed=4200 + i, dtype="f32", stretch=s)
             for i, (n, nz, s) in enumerate(SMALL[:3])]
    batch = BatchPlan([p.grid for p in probs], precision="fp32", lanes=2)
    host = [torch.from_numpy(p.rhs_as("f32")) for p in probs]
    rhs = [torch.zeros_like(h, device="cuda") for h in host]
    out = [torch.empty_like(r) for r in rhs]
    batch.solve(rhs, out)  # capture with these pointers
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for r, h in zip(rhs, host):
            r.copy_(h.cuda(non_blocking=False))
            r.mul_(2.0)
        batch.solve(rhs, out)
        copies = [o.clone() for o in out]
    s.synchronize()
    ref = standalone([p.grid for p in probs], [2 * h.cuda() for h in host], "fp32")
    for c, r in zip(copies, ref):
        assert torch.equal(c, r)
    batch.close()


def test_batch_rejects_withdrawn_modes_and_bad_lanes():
    from paper_2010_14132_amd import BatchPlan
    from paper_2010_14132_amd.binding import PressureSolveError
    g = wl.stretched_smooth(32, 32, 8, seed=1, dtype="f32").grid
    for mode in ("phases", "persistent", "plans"):
        with pytest.raises(PressureSolveError):
            BatchPlan([g], precision="fp32", mode=mode)
    batch = BatchPlan([g], precision="fp32")
    for bad in (0, 9, -1):
        with pytest.raises(PressureSolveError):
            batch.set_lanes(bad)
    from paper_2010_14132_amd.binding import load
    for bad in (2, -1):
        assert load().ps_batch_set_fp64_order(batch._h, bad) == 1  # PS_EINVAL
    assert batch.info()["fp64_in_order"]
    batch.close()


def test_full_uneven_batch_48():
    """The 48-problem recipe (nx = ny from {64..512} incl. 3*2^k sizes, nz
    from {32..128}, stretching in [1, 1.05], seed 4), FP32, autotuned as
    the benchmark runs it: every problem equal to its standalone autotuned
    plan, and against the oracle (whole field up to 2^20 points, sampled
    wavenumber columns above).  Replay time reported."""
    from paper_2010_14132_amd import BatchPlan
    probs = wl.batch_problems()
    npts = sum(p.grid.points for p in probs)
    announce("batch of 48 uneven problems, %d points" % npts)
    batch = BatchPlan([p.grid for p in probs], precision="fp32")
    rhs = [torch.from_numpy(p.rhs_as("f32")).cuda() for p in probs]
    out = [torch.empty_like(r) for r in rhs]
    batch.autotune(rhs, out, reps=3)
    info = batch.info()
    announce("autotuned: %d lanes, FP64 columns %s"
             % (info["lanes"], "in order" if info["fp64_in_order"] else "forked"))
    for o in out:
        o.zero_()
    batch.solve(rhs, out)
    batch.status()
    single = standalone([p.grid for p in probs], rhs, "fp32", autotune=True)
    for i in range(len(probs)):
        assert torch.equal(out[i], single[i]), (i, probs[i].grid.nx, probs[i].grid.nz)
    del single
    announce("48 problems bit-equal to their standalone plans; oracle checks")
    check_oracle(probs, out, 1e-5)

    def per_call(fn, n=20):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / n * 1e3

    ms = per_call(lambda: batch.solve(rhs, out))
    print("48 problems: %.3f ms per batched solve, %.0f Mpts/s" % (ms, npts / ms / 1e3))
    batch.close()
