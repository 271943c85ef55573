"""Solves in MONC's own field layout p%data(z,y,x) (z fastest, a C array
[nx][ny][nz]) through ps_solve_zyx.  Register-resident lengths go through a
[kx][j][k] buffer (x and y passes staging along k); other lengths through x
passes that transpose in LDS around the level-major y and column passes.
Either way the row transforms are the level-major solve's: with the
generic x passes the two layouts give the same bits, with the register-
resident ones they agree to rounding; both against the oracle."""
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


def grid(nx, ny, nz, seed):
    r = np.random.default_rng(seed)
    g = wl.stretched_grid(nx, ny, nz, stretch=1.03)
    g.dz = g.dz * r.uniform(0.8, 1.2, nz)
    g.dy = 37.0
    return g


SHAPES = [(16, 32, 64), (5, 12, 18), (1, 8, 8), (33, 1, 16), (128, 24, 48), (7, 27, 54),
          (64, 64, 256), (9, 16, 1024)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_r2"])
def test_zyx_solve_matches_level_major_and_oracle(tmp_path, precision, shape):
    from paper_2010_14132_amd import Plan
    from paper_2010_14132_amd.binding import PRECISIONS, tune_cache_load
    nz, ny, nx = shape
    announce("zyx solve %s %s" % (precision, shape))
    g = grid(nx, ny, nz, seed=nz + ny + nx)
    b = np.random.default_rng(5).standard_normal(shape) + 0.3
    dt = torch.float64 if precision == "fp64" else torch.float32
    if precision != "fp64":
        b = b.astype(np.float32).astype(np.float64)
    # the generic x transforms for the level-major plan (x, y, columns, beside,
    # chunks, backward x); the tile split of the z-fastest passes varies
    for kc in (1, 4, 64):
        f = tmp_path / ("tune%d.txt" % kc)
        f.write_text("%s %d %d %d %d 0 1 3 1 1 0 1 %d\n"
                     % (arch(), nx, ny, nz, PRECISIONS[precision], kc))
        tune_cache_load(str(f))
        plan = Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.rho, precision=precision)
        plan.autotune()
        assert plan.info()["zyx_kc"] == kc
        bt = torch.from_numpy(b).to("cuda", dt)
        bz = bt.permute(2, 1, 0).contiguous()          # [nx][ny][nz]
        p_lm = plan.solve(bt)
        p_z = plan.solve_zyx(bz)
        l_lm = plan.solve_adjoint(bt)
        l_z = plan.solve_zyx(bz, adjoint=True)
        torch.cuda.synchronize()
        assert torch.equal(p_z.permute(2, 1, 0), p_lm), kc
        assert torch.equal(l_z.permute(2, 1, 0), l_lm), kc
        plan.close()
    ref = oracle.solve(b, g.dx, g.dy, g.dz, g.rho)
    lref = oracle.solve_adjoint(b, g.dx, g.dy, g.dz, g.rho)
    assert relmax(p_z.permute(2, 1, 0).double().cpu().numpy(), ref) < TOL[precision]
    assert relmax(l_z.permute(2, 1, 0).double().cpu().numpy(), lref) < TOL[precision]


FAST_SHAPES = [(16, 32, 64), (1, 16, 32), (33, 64, 256), (9, 16, 1024), (70, 64, 32),
               (5, 128, 512), (3, 1024, 32), (20, 64, 128), (36, 16, 256), (12, 96, 192)]


@pytest.mark.parametrize("shape", FAST_SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_r2"])
def test_zyx_fast_passes_bit_equal_to_level_major(tmp_path, precision, shape):
    """Register-resident lengths: the z-fastest solve through the [kx][j][k]
    buffer (x passes staging along k, y passes between that buffer and the
    spectrum) runs the same row transforms as the level-major solve with
    the same variants (plain and paired x, both y tile orders, standard and
    wide blocks of levels); the compiler
    fuses a few products differently in the separately built kernels, so
    the two agree to rounding (not bit for bit), forward and adjoint, and
    each is checked against the oracle; the in-place call gives the same
    bits as the out-of-place one.  Partial level chunks (nz not a multiple
    of a block's levels) and nz = 1 included."""
    from paper_2010_14132_amd import Plan
    from paper_2010_14132_amd.binding import PRECISIONS, tune_cache_load
    nz, ny, nx = shape
    announce("zyx fast passes %s %s" % (precision, shape))
    g = grid(nx, ny, nz, seed=nz + 2 * ny + nx)
    b = np.random.default_rng(6).standard_normal(shape) + 0.3
    dt = torch.float64 if precision == "fp64" else torch.float32
    if precision != "fp64":
        b = b.astype(np.float32).astype(np.float64)
    ref = oracle.solve(b, g.dx, g.dy, g.dz, g.rho)
    lref = oracle.solve_adjoint(b, g.dx, g.dy, g.dz, g.rho)
    # plain x with the standard blocks, paired x with the wide blocks
    for vx, vy, kc in ((1, 1, 16), (4, 2, 64)):
        f = tmp_path / ("tune%d.txt" % vx)
        f.write_text("%s %d %d %d %d %d %d 3 1 1 %d 1 %d\n"
                     % (arch(), nx, ny, nz, PRECISIONS[precision], vx, vy, vx, kc))
        tune_cache_load(str(f))
        plan = Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.rho, precision=precision)
        plan.autotune()
        info = plan.info()
        assert (info["fft_variant_x"], info["fft_variant_y"], info["fft_variant_xi"]) == (vx, vy, vx)
        bt = torch.from_numpy(b).to("cuda", dt)
        bz = bt.permute(2, 1, 0).contiguous()          # [nx][ny][nz]
        p_lm = plan.solve(bt)
        p_z = plan.solve_zyx(bz)
        l_lm = plan.solve_adjoint(bt)
        l_z = plan.solve_zyx(bz, adjoint=True)
        x = bz.clone()
        plan.solve_zyx(x, out=x)
        torch.cuda.synchronize()
        agree = 1e-14 if precision == "fp64" else 2e-6
        pz, lz = p_z.permute(2, 1, 0).double().cpu().numpy(), l_z.permute(2, 1, 0).double().cpu().numpy()
        assert relmax(pz, p_lm.double().cpu().numpy()) < agree, (vx, vy)
        assert relmax(lz, l_lm.double().cpu().numpy()) < agree, (vx, vy)
        assert torch.equal(x, p_z), (vx, vy)
        assert plan.workspace_bytes() >= 2 * nz * ny * (nx // 2) * (16 if precision == "fp64" else 8)
        plan.close()
        assert relmax(pz, ref) < TOL[precision], (vx, vy)
        assert relmax(lz, lref) < TOL[precision], (vx, vy)


def test_zyx_in_place_and_r1_aliasing_refused():
    from paper_2010_14132_amd import Plan
    from paper_2010_14132_amd.binding import PressureSolveError
    g = grid(32, 24, 10, seed=3)
    b = torch.from_numpy(np.random.default_rng(2).standard_normal((32, 24, 10))).cuda()
    plan = Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.rho, precision="fp64")
    want = plan.solve_zyx(b)
    x = b.clone()
    plan.solve_zyx(x, out=x)
    torch.cuda.synchronize()
    assert torch.equal(x, want)
    plan.close()
    plan = Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.rho, precision="fp32_r1")
    x = b.float()
    with pytest.raises(PressureSolveError):
        plan.solve_zyx(x, out=x)  # the refinement reads the right-hand side after p exists
    plan.close()


R1_SHAPES = [(16, 32, 64), (5, 12, 18), (1, 8, 8), (33, 64, 256), (12, 96, 192),
             (7, 16, 1024), (128, 24, 48)]


@pytest.mark.parametrize("shape", R1_SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_zyx_refinement_r1(shape):
    """The FP32 form with one physical-residual refinement step in the
    z-fastest layout (residual pass of its own, correction accumulated by
    the last backward x pass), forward and adjoint: against the oracle at
    the refinement's bar, and against the level-major refined solve; the
    register-resident and the generic passes both (shapes of either kind)."""
    from paper_2010_14132_amd import Plan
    nz, ny, nx = shape
    announce("zyx fp32_r1 %s" % (shape,))
    g = grid(nx, ny, nz, seed=nz + 3 * ny + nx)
    b = np.random.default_rng(9).standard_normal(shape).astype(np.float32).astype(np.float64) + 0.3
    plan = Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.rho, precision="fp32_r1")
    bt = torch.from_numpy(b).to("cuda", torch.float32)
    bz = bt.permute(2, 1, 0).contiguous()
    p_z = plan.solve_zyx(bz).permute(2, 1, 0).double().cpu().numpy()
    l_z = plan.solve_zyx(bz, adjoint=True).permute(2, 1, 0).double().cpu().numpy()
    p_lm = plan.solve(bt).double().cpu().numpy()
    plan.close()
    ref = oracle.solve(b, g.dx, g.dy, g.dz, g.rho)
    lref = oracle.solve_adjoint(b, g.dx, g.dy, g.dz, g.rho)
    e, el, d = relmax(p_z, ref), relmax(l_z, lref), relmax(p_z, p_lm)
    print("zyx fp32_r1 %s: forward %.2e adjoint %.2e vs level-major %.2e" % (shape, e, el, d))
    assert e < TOL["fp32_r1"] and el < TOL["fp32_r1"] and d < 2 * TOL["fp32_r1"]


def test_zyx_autotuned_1024_sampled():
    """The precision workload at 1024^2 x 128 in the z-fastest layout,
    autotuned (the tile split included): equal to the level-major autotuned
    solve to FP32 rounding of the transforms, and sampled wavenumber columns
    against the oracle's column solves."""
    from paper_2010_14132_amd import Plan
    from tests import sampling
    prob = wl.precision_1024("f32")
    g = prob.grid
    announce("zyx 1024^2x128 fp32_r2 autotuned")
    plan = Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.rho, precision="fp32_r2")
    plan.autotune(reps=3)
    bt = torch.from_numpy(prob.rhs_as("f32")).cuda()
    pz = plan.solve_zyx(bt.permute(2, 1, 0).contiguous()).permute(2, 1, 0)
    plm = plan.solve(bt)
    torch.cuda.synchronize()
    d = ((pz - plm).abs().max() / plm.abs().max()).item()
    print("zyx vs level-major rel_max %.3e, zyx_kc %d" % (d, plan.info()["zyx_kc"]))
    assert d < 1e-5
    p = pz.double().cpu().numpy()
    b = prob.rhs_exact()
    scale, errs = 0.0, []
    for kx, ky in [(1, 0), (0, 1), (3, 7), (100, 200)]:
        want = sampling.forward_column(b, kx, ky, g.dx, g.dy, g.dz, g.rho)
        got = sampling.dft_at(p, kx, ky)
        scale = max(scale, np.abs(want).max())
        errs.append(np.abs(got - want).max())
    assert max(errs) / scale < 1e-5
    plan.close()
