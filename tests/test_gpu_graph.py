"""Solves captured into a HIP graph by the caller (torch.cuda.graph).

The solve path only launches kernels and records and waits on events (the
FP64 columns fork onto the plan's second stream and join back), so a caller
can capture it.  Every replay runs on a new input, with eager solves and
synchronisations between replays, and must reproduce the eager result bit
for bit (same kernels, same order, no atomics); one replay is also checked
against the oracle.
"""
import time

import numpy as np
import pytest

import oracle
from paper_2010_14132_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NZ, NY, NX = 16, 64, 128


def announce(msg):
    print("\n[gpu] " + msg, flush=True)


def grid():
    g = wl.stretched_grid(NX, NY, NZ)
    g.dy = 37.0
    return g


def make_plan(g, precision):
    from paper_2010_14132_amd import Plan
    return Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.rho, precision=precision)


def field(seed, dtype):
    b = np.random.default_rng(seed).standard_normal((NZ, NY, NX)) + 0.2
    return torch.from_numpy(b).to("cuda", dtype)


def capture(fn):
    """Warm up on a side stream (default priority), then capture fn."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fn()
    torch.cuda.synchronize()
    return graph


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_r2", "fp32_r1"])
def test_solve_graph_replays_match_eager(precision):
    announce("graph-captured solve %s %dx%dx%d" % (precision, NZ, NY, NX))
    g = grid()
    plan = make_plan(g, precision)
    dt = torch.float64 if precision == "fp64" else torch.float32
    static_b = field(0, dt)
    static_out = torch.empty_like(static_b)
    graph = capture(lambda: plan.solve(static_b, out=static_out))
    for rep in range(4):
        b = field(100 + rep, dt)
        static_b.copy_(b)
        graph.replay()
        torch.cuda.synchronize()
        eager = plan.solve(b)
        torch.cuda.synchronize()
        assert torch.equal(static_out, eager), "replay %d differs from the eager solve" % rep
        if rep == 1:
            bb = b.cpu().numpy().astype(np.float64)
            ref = oracle.solve(bb, g.dx, g.dy, g.dz, g.rho)
            err = np.abs(static_out.cpu().numpy() - ref).max() / np.abs(ref).max()
            assert err < (1e-12 if precision == "fp64" else 1e-5)
    plan.close()


@pytest.mark.parametrize("side", [0, 1, 2])
@pytest.mark.parametrize("precision", ["fp64", "fp32_r2", "fp32_r1"])
def test_level_range_solve_graph(tmp_path, precision, side):
    """A solve whose x and y passes run over 3 level ranges (the tune cache's
    xy_chunks), with each FP64-column placement -- with placement 1 the
    second stream waits on an event re-recorded after every range's x pass
    -- captured into a graph and replayed against eager solves."""
    from paper_2010_14132_amd.binding import PRECISIONS, tune_cache_load
    announce("graph-captured level-range solve %s side %d" % (precision, side))
    g = grid()
    f = tmp_path / "tune.txt"
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    f.write_text("%s %d %d %d %d 1 1 3 %d 1 1 1 64 3\n"
                 % (arch, NX, NY, NZ, PRECISIONS[precision], side))
    tune_cache_load(str(f))
    plan = make_plan(g, precision)
    plan.autotune()
    assert plan.info()["xy_chunks"] == 3 and plan.info()["fp64_beside"] == side
    dt = torch.float64 if precision == "fp64" else torch.float32
    static_b = field(5, dt)
    static_out = torch.empty_like(static_b)
    graph = capture(lambda: plan.solve(static_b, out=static_out))
    for rep in range(3):
        b = field(400 + rep, dt)
        static_b.copy_(b)
        graph.replay()
        torch.cuda.synchronize()
        eager = plan.solve(b)
        torch.cuda.synchronize()
        assert torch.equal(static_out, eager), "replay %d differs from the eager solve" % rep
    plan.close()


def test_differentiation_step_graph():
    """Solve, adjoint solve and density gradient in one captured graph
    (FP32 + in-register refinement), replayed against the eager calls."""
    announce("graph-captured solve + adjoint + grad fp32_r2")
    g = grid()
    plan = make_plan(g, "fp32_r2")
    b, w = field(1, torch.float32), field(2, torch.float32)
    p, lam = torch.empty_like(b), torch.empty_like(b)
    grho = torch.empty(NZ, dtype=torch.float64, device="cuda")

    def step():
        plan.solve(b, out=p)
        plan.solve_adjoint(w, out=lam)
        grho.copy_(plan.grad_coeffs(lam, p))

    graph = capture(step)
    for rep in range(3):
        nb, nw = field(200 + rep, torch.float32), field(300 + rep, torch.float32)
        b.copy_(nb)
        w.copy_(nw)
        graph.replay()
        torch.cuda.synchronize()
        ep = plan.solve(nb)
        el = plan.solve_adjoint(nw)
        eg = plan.grad_coeffs(el, ep)
        torch.cuda.synchronize()
        assert torch.equal(p, ep) and torch.equal(lam, el) and torch.equal(grho, eg), rep
    plan.close()


@pytest.mark.parametrize("precision", ["fp32_r2", "fp32_r1", "fp64"])
def test_zyx_and_projection_graphs(precision):
    """A z-fastest solve (its buffers allocated by the warm-up call) and a
    projection step with the gradient correction, each captured and
    replayed on new inputs, bit-equal to the eager calls."""
    announce("graph-captured z-fastest solve and projection step %s" % precision)
    g = grid()
    plan = make_plan(g, precision)
    dt = torch.float64 if precision == "fp64" else torch.float32
    bz = field(3, dt).permute(2, 1, 0).contiguous()
    pz = torch.empty_like(bz)
    gz = capture(lambda: plan.solve_zyx(bz, out=pz))
    u, v, w = field(4, dt), field(5, dt), field(6, dt)
    pp = torch.empty_like(u)
    gp = capture(lambda: plan.project(u, v, w, 2.0, out=pp, correct=True))
    for rep in range(3):
        nb = field(400 + rep, dt).permute(2, 1, 0).contiguous()
        bz.copy_(nb)
        gz.replay()
        nu, nv, nw = field(500 + rep, dt), field(600 + rep, dt), field(700 + rep, dt)
        u.copy_(nu)
        v.copy_(nv)
        w.copy_(nw)
        gp.replay()
        torch.cuda.synchronize()
        ez = plan.solve_zyx(nb)
        ep = plan.project(nu, nv, nw, 2.0, correct=True)
        torch.cuda.synchronize()
        assert torch.equal(pz, ez), rep
        assert torch.equal(pp, ep) and torch.equal(u, nu) and torch.equal(v, nv) \
            and torch.equal(w, nw), rep
    plan.close()


def test_graph_replay_launch_time_small_grid():
    """At 64 x 128 x 16 a solve is a few tens of microseconds, comparable
    with the launches it issues; replaying a captured graph removes their
    host cost.  Reported, not asserted beyond correctness."""
    announce("graph replay vs eager timing fp32_r2 %dx%dx%d" % (NZ, NY, NX))
    g = grid()
    plan = make_plan(g, "fp32_r2")
    b = field(3, torch.float32)
    out = torch.empty_like(b)
    graph = capture(lambda: plan.solve(b, out=out))

    def per_call(fn, n=200):
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / n * 1e6

    eager_us = per_call(lambda: plan.solve(b, out=out))
    graph_us = per_call(graph.replay)
    print("eager %.1f us/solve, graph replay %.1f us/solve" % (eager_us, graph_us))
    ref = plan.solve(b)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    plan.close()
