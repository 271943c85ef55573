"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every entry point include/pressure_solve.h declares, and argument
validation rejects bad input before any HIP call."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pressure_solve.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ps_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2010_14132_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libpressure_solve.so is not built; run __graft_entry__.build()")
    return binding.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("ps_plan_create", "ps_solve", "ps_solve_adjoint", "ps_grad_coeffs",
                 "ps_batch_create", "ps_batch_solve", "ps_plan_destroy"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2010_14132_amd import binding
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in binding.SIGNATURES, "binding lacks " + name


def _create(lib, nx=32, ny=32, nz=16, dx=50.0, dy=50.0, dz=None, rho=None, prec=0, tau=0.0):
    from paper_2010_14132_amd import binding
    dz = np.full(nz, 40.0) if dz is None else np.asarray(dz, dtype=np.float64)
    rho = np.ones(nz) if rho is None else np.asarray(rho, dtype=np.float64)
    h = ctypes.c_void_p(12345)
    rc = lib.ps_plan_create(ctypes.byref(h), nx, ny, nz, dx, dy, binding._dptr(dz),
                            binding._dptr(rho), prec, tau, None)
    return rc, h


@pytest.mark.parametrize("kw,code", [
    (dict(nx=31), 2), (dict(nx=0), 2), (dict(nx=2 * 5 * 7), 2), (dict(nx=4096), 2),
    (dict(ny=0), 2), (dict(ny=10), 2), (dict(ny=2048), 2),
    (dict(nz=0), 2), (dict(nz=257, dz=np.full(257, 1.0), rho=np.ones(257)), 2),
    (dict(dx=0.0), 1), (dict(dy=-1.0), 1), (dict(dx=math.inf), 1), (dict(dx=math.nan), 1),
    (dict(dz=[40.0] * 15 + [0.0]), 1), (dict(rho=[1.0] * 15 + [-1.0]), 1),
    (dict(rho=[1.0] * 15 + [math.nan]), 1), (dict(prec=7), 2), (dict(prec=-1), 2),
    (dict(tau=math.nan), 1),
])
def test_create_rejects_bad_arguments_before_any_hip_call(lib, kw, code):
    rc, h = _create(lib, **kw)
    assert rc == code, (kw, rc, lib.ps_last_error())
    assert h.value is None  # *out is cleared on error


def test_null_arguments(lib):
    assert lib.ps_plan_create(None, 32, 32, 16, 50.0, 50.0, None, None, 0, 0.0, None) == 1
    assert lib.ps_solve(None, None, None) == 1
    assert lib.ps_solve_adjoint(None, None, None) == 1
    assert lib.ps_grad_coeffs(None, None, None, None) == 1
    assert lib.ps_plan_set_coeffs(None, None) == 1
    assert lib.ps_plan_query(None, None) == 1
    assert lib.ps_forward_transform(None, None, None) == 1
    assert lib.ps_spectral_solve(None, None, 0) == 1
    assert lib.ps_inverse_transform(None, None, None) == 1
    assert lib.ps_plan_destroy(None) == 0
    assert lib.ps_workspace_bytes(None) == 0
    assert lib.ps_plan_profile(None, 1) == 1
    assert lib.ps_plan_profile_report(None, 0, None, None, None) == 1


def test_status_strings(lib):
    for s in range(6):
        assert lib.ps_status_string(s)
    assert lib.ps_status_string(99) == b"unknown status"
    rc, _ = _create(lib, nx=31)
    assert b"nx" in lib.ps_last_error()


def test_tune_cache_round_trip_and_rejects_bad_lines(lib, tmp_path):
    """The tune-cache text format (host-only code): full and short lines are
    read with their defaults, malformed or out-of-range lines are skipped,
    and a save writes every entry back with all fields."""
    src = tmp_path / "in.txt"
    src.write_text("\n".join([
        "gfx950 512 256 64 1 2 1 5 1 4 3 0 8", # every field
        "gfx950 96 96 16 1 1 1 3 1 1 1 1 0",  # z-fastest tile levels out of range
        "gfx950 128 128 16 1 1 1 3 1 1 1 2", # FP64-column variant out of range
        "gfx950 256 256 32 0 1 1 3",         # short: fp64_beside 1, chunks 1, xi = x
        "gfx950 256 256 32 2 1 1 7 2",       # FP64 columns forked after the y pass
        "gfx950 512 512 32 2 1 1 7 3",       # fp64_beside out of range
        "gfx950 64 64 8 2 9 1 3",            # x variant out of range
        "gfx950 64 64 8 3 1 1 9",            # column variant out of range
        "gfx950 64 64 8 1 1 1 3 1 0",        # chunks out of range
        "gfx950 1024 1024 128 2 4 1 7 2 1 1 1 16 2",  # level ranges of the x / y passes
        "gfx950 1024 1024 128 1 4 1 4 2 1 1 1 16 0",  # xy_chunks out of range
        "not a line",
        "",
    ]) + "\n")
    assert lib.ps_tune_cache_load(os.fsencode(str(src))) == 0
    out = tmp_path / "out.txt"
    assert lib.ps_tune_cache_save(os.fsencode(str(out))) == 0
    lines = {tuple(l.split()[:5]): l.split()[5:] for l in out.read_text().splitlines() if l}
    assert lines[("gfx950", "512", "256", "64", "1")] == ["2", "1", "5", "1", "4", "3", "0", "8", "1"]
    assert lines[("gfx950", "256", "256", "32", "0")] == ["1", "1", "3", "1", "1", "1", "1", "64", "1"]
    assert lines[("gfx950", "256", "256", "32", "2")] == ["1", "1", "7", "2", "1", "1", "1", "64", "1"]
    assert lines[("gfx950", "1024", "1024", "128", "2")] == ["4", "1", "7", "2", "1", "1", "1", "16", "2"]
    assert ("gfx950", "1024", "1024", "128", "1") not in lines
    assert ("gfx950", "512", "512", "32", "2") not in lines
    assert ("gfx950", "96", "96", "16", "1") not in lines
    assert ("gfx950", "128", "128", "16", "1") not in lines
    assert not any(k[1:4] == ("64", "64", "8") for k in lines)
    assert lib.ps_tune_cache_load(os.fsencode(str(tmp_path / "missing.txt"))) == 1


def test_new_entry_points_reject_bad_arguments_before_any_hip_call(lib):
    """Batched, conjugate-gradient, z-fastest, projection and no-allocation
    entry points validate on the host (no GPU needed)."""
    from paper_2010_14132_amd import binding
    vp = ctypes.c_void_p
    one = (ctypes.c_int * 1)(8)
    d1 = (ctypes.c_double * 1)(50.0)
    dz = np.full(8, 40.0)
    arr = (binding._D * 1)(binding._dptr(dz))
    h = vp(1234)
    assert lib.ps_batch_create(None, 1, one, one, one, d1, d1, arr, arr, 1, None) == 1
    assert lib.ps_batch_create(ctypes.byref(h), 0, one, one, one, d1, d1, arr, arr, 1, None) == 1
    assert h.value is None
    assert lib.ps_batch_create(ctypes.byref(h), 1, None, one, one, d1, d1, arr, arr, 1, None) == 1
    assert lib.ps_batch_create(ctypes.byref(h), 1, one, one, one, d1, d1, arr, arr, 9, None) == 2
    nul = (binding._D * 1)()
    assert lib.ps_batch_create(ctypes.byref(h), 1, one, one, one, d1, d1, nul, arr, 1, None) == 1
    assert lib.ps_batch_solve(None, None, None) == 1
    assert lib.ps_batch_set_lanes(None, 2) == 1
    assert lib.ps_batch_set_mode(None, 3) == 1
    assert lib.ps_batch_autotune(None, None, None, 1) == 1
    assert lib.ps_batch_query(None, None, None, None) == 1
    assert lib.ps_batch_set_fp64_order(None, 1) == 1
    assert lib.ps_batch_status(None) == 1
    assert lib.ps_batch_destroy(None) == 0
    rho = np.ones(8)
    for args, code in (((8, 8, 8, 50.0, 50.0, binding._dptr(dz), binding._dptr(rho), 7), 1),
                       ((0, 8, 8, 50.0, 50.0, binding._dptr(dz), binding._dptr(rho), 1), 2),
                       ((8, 8, 8, -1.0, 50.0, binding._dptr(dz), binding._dptr(rho), 1), 1),
                       ((8, 8, 8, 50.0, 50.0, None, binding._dptr(rho), 1), 1),
                       ((1 << 12, 1 << 12, 1 << 8, 50.0, 50.0, binding._dptr(dz),
                         binding._dptr(rho), 1), 2)):
        assert lib.ps_cg_create(ctypes.byref(h), *args, None) == code, args
        assert h.value is None
    bad = np.full(8, 40.0)
    bad[3] = -1.0
    assert lib.ps_cg_create(ctypes.byref(h), 8, 8, 8, 50.0, 50.0, binding._dptr(bad),
                            binding._dptr(rho), 1, None) == 1
    assert lib.ps_cg_solve(None, None, None, 1e-6, 10, None, None) == 1
    assert lib.ps_cg_set_method(None, 1) == 1
    assert lib.ps_cg_destroy(None) == 0
    assert lib.ps_cg_workspace_bytes(None) == 0
    assert lib.ps_solve_zyx(None, None, None, 0) == 1
    assert lib.ps_project(None, None, None, None, 1.0, None, 1) == 1
    assert lib.ps_grad_coeffs_noalloc(None, None, None, None) == 1
