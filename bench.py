#!/usr/bin/env python3
"""Benchmark of the direct FFT pressure solve on one MI355X.

Workload: 1024 x 1024 x 128 stretched grid (dz_k = 20 m * 1.03^k, dx = dy =
50 m), density rho(z) = exp(-z / 8000 m), smooth k^-2 right-hand side plus
1 % white noise (seed 2) -- the precision-form configuration the headline
metric is quoted on.  A step is one complete solve (forward transforms,
column solves, backward transforms and the refinement) of that right-hand
side, already resident in HBM.

Prints ONE JSON line: the headline value is solves/s of the FP32 form with
refinement (precision "fp32_r2" by default), with the plain FP64 GPU solve
and the other precision forms measured on the same grid beside it, the
roofline of the dominant kernel, the whole solve's share of HBM peak, the
other workloads (32^2 x 16 plain, 256^2 x 64 plain, 512^2 x 128
differentiation, the 48-problem uneven batch) under "configs", and on the
CPU side the oracle timed on a bounded sample (all cores, and one core for
the two small workloads) next to a fast FP64 CPU solve (scipy FFTs and a
vectorised column sweep), which is labelled apart from the oracle.  The
oracle runs only in the CPU baseline (timing); errors are reported against
the FP64 GPU solve, whose parity with the oracle the GPU tests check.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure

# Algorithmic HBM bytes per grid point of each kernel, for element size e
# (4 for FP32, 8 for FP64).  The spectrum holds nz * (nx/2) * ny complex
# values = N/2 complex = N e bytes; real fields hold N e bytes.
#   fwd_x:     read real field (N e) + write spectrum (N e)        = 2e per point
#   fft_y_*:   read + write spectrum                               = 2e
#   columns:   read + write the spectrum of the kx >= 1 columns    = 2e (1 - 2/nx)
#   inv_x:     read spectrum + write real field                    = 2e
#   fwd_x_residual: read b, read p, write spectrum                 = 3e
#   inv_x with accumulation (refinement): + read p                 = 3e




def kernel_bytes_per_point(name: str, e: int, nx: int, accumulate: bool = False) -> float:
    if name == "columns":
        return 2.0 * e * (1.0 - 2.0 / nx)
    if name == "fwd_x_residual":
        return 3.0 * e
    if name == "inv_x" and accumulate:
        return 3.0 * e
    return {"fwd_x": 2.0 * e, "fft_y_fwd": 2.0 * e, "fft_y_inv": 2.0 * e,
            "inv_x": 2.0 * e}.get(name, 0.0)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_solve_1024x1024x128.txt")


def kernel_sources_digest() -> str:
    """SHA-256 (first 16 hex digits) of the HIP sources, in name order: a
    counter summary taken on other sources no longer describes the kernels."""
    import hashlib
    d = os.path.join(ROOT, "paper_2010_14132_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".h")):
            h.update(name.encode())
            with open(os.path.join(d, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(form: str, kernel: str):
    """HBM bytes per solve (FETCH_SIZE + WRITE_SIZE, each scaled by the
    factor a plain device copy of known size gives) of one kernel of one
    precision form, from the committed rocprofv3 counter summary, or None if
    there is none for it or it was taken on other kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    digest, found = None, None
    with open(TRAFFIC_FILE) as f:
        for line in f:
            w = line.split()
            if len(w) >= 2 and w[0] == "sources":
                digest = w[1]
            if len(w) >= 4 and w[0] == "form" and w[1] == form and w[2] == "kernel" and w[3] == kernel:
                kv = dict(zip(w[4::2], w[5::2]))
                found = float(kv["fetch_bytes_per_solve"]) + float(kv["write_bytes_per_solve"])
    if digest != kernel_sources_digest():
        return None
    return found


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, nz_full: int):
    """Time the FP64 oracle (as it stands) on a bounded sample of the same
    workload: the full 1024 x 1024 horizontal grid with three levels per oracle
    thread (its parallel loop runs over levels), same recipe.  The oracle's
    cost per point does not depend on nz (direct DFTs per level dominate),
    so the full-size time is scaled by nz_full / levels."""
    import oracle
    from paper_2010_14132_amd import workloads as wl
    threads = oracle.num_threads()
    levels = int(min(max(3 * threads, 8), 96))  # three levels per thread: ~12 s on 16 cores
    sg = wl.stretched_grid(g.nx, g.ny, levels)
    b = wl.smooth_field(np.random.default_rng(2), sg, noise=0.01)
    t0 = time.perf_counter()
    oracle.solve(b, sg.dx, sg.dy, sg.dz, sg.rho)
    t = time.perf_counter() - t0
    t_full = t * nz_full / levels
    return {"value": 1.0 / t_full, "unit": "solves/s", "cores": min(threads, levels),
            "kind": "oracle",
            "sample": "FP64 oracle solve of %dx%dx%d levels of the same recipe in %.2f s, "
                      "scaled by %d/%d levels to %.1f s per full solve"
                      % (g.nx, g.ny, levels, t, nz_full, levels, t_full),
            "mpts_per_s": g.nx * g.ny * nz_full / t_full / 1e6, "cpu_model": cpu_model()}


def time_calls(call, steps, warmup):
    """Mean ms per call of `call` (work enqueued on the current stream),
    after `warmup` untimed calls."""
    import torch
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(steps):
        call()
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def time_solves(plan, b, out, steps, warmup):
    return time_calls(lambda: plan.solve(b, out=out), steps, warmup)


def time_distribution(call, reps):
    """Per-call device times (ms) of `reps` calls, each bracketed by its own
    pair of events on the current stream: (median, min, mean)."""
    import torch
    st = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record(st)
        call()
        b.record(st)
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in ev])
    return {"median_ms": float(np.median(t)), "min_ms": float(t.min()),
            "mean_ms": float(t.mean()), "reps": reps}


# ------------------------------------------------------------ fast CPU reference
def fast_cpu_solve(b, dx, dy, dz, rho, workers):
    """The same discrete problem solved on the CPU in FP64 the fast way, as a
    speed reference next to the oracle (whose direct DFTs make it slow): the
    D-weighted mean removed, scipy.fft real 2D transforms of all levels with
    `workers` threads, the dominance-excess column sweep vectorised over all
    wavenumbers (numpy), the mean column by flux prefix sums with the
    zero-mean gauge, and the inverse transform."""
    import scipy.fft as sfft
    b = np.asarray(b, dtype=np.float64)
    nz, ny, nx = b.shape
    dz = np.asarray(dz, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    f = np.zeros(nz + 1)                       # f[k] = f_{k-1/2}, zero at both ends
    f[1:nz] = 0.5 * (rho[:-1] + rho[1:]) / (0.5 * (dz[:-1] + dz[1:]))
    D = rho * dz
    S = b.sum(axis=(1, 2))
    mu = float((D * S).sum() / (nx * ny * D.sum()))
    B = sfft.rfft2(b, axes=(1, 2), workers=workers)   # [nz][ny][nx/2+1]
    B[:, 0, 0] -= mu * nx * ny
    kx = np.arange(nx // 2 + 1)
    ky = np.arange(ny)
    s = (4 * np.sin(np.pi * ky / ny) ** 2 / dy ** 2)[:, None] \
        + (4 * np.sin(np.pi * kx / nx) ** 2 / dx ** 2)[None, :]
    mean_col = B[:, 0, 0].real.copy()
    s[0, 0] = 1.0                               # placeholder: the mean column is done apart
    # forward elimination of (-D T) x = -D b_hat, pivots u_k from positive terms
    U = np.empty((nz,) + s.shape)
    eps = s * D[0]
    U[0] = eps + f[1]
    B[0] *= -D[0]
    for k in range(1, nz):
        g = f[k] / U[k - 1]
        eps = s * D[k] + g * eps
        U[k] = eps + f[k + 1]
        B[k] *= -D[k]
        B[k] += g * B[k - 1]
    B[nz - 1] /= U[nz - 1]
    for k in range(nz - 2, -1, -1):
        B[k] += f[k + 1] * B[k + 1]
        B[k] /= U[k]
    # mean column: V x = c by flux prefix sums, then zero mean over levels
    x = np.zeros(nz)
    flux = 0.0
    for k in range(nz - 1):
        flux += D[k] * mean_col[k]
        x[k + 1] = x[k] + flux / f[k + 1]
    B[:, 0, 0] = x - x.mean()
    return sfft.irfft2(B, s=(ny, nx), axes=(1, 2), workers=workers)


def fast_cpu_reference(prob, p_gpu64=None):
    """Times fast_cpu_solve on the full workload with every host core (the
    better of two runs) and, given the FP64 GPU solution, reports the two
    solutions' relative difference."""
    g = prob.grid
    workers = os.cpu_count() or 1
    b = prob.rhs_exact()
    best = None
    for _ in range(2):
        t0 = time.perf_counter()
        p = fast_cpu_solve(b, g.dx, g.dy, g.dz, g.rho, workers)
        t = time.perf_counter() - t0
        best = t if best is None else min(best, t)
    out = {"kind": "fast_cpu_reference (not the oracle)", "value": 1.0 / best,
           "unit": "solves/s", "ms_per_solve": best * 1e3, "cores": workers,
           "mpts_per_s": g.points / best / 1e6,
           "method": "FP64: scipy.fft rfft2/irfft2 over all levels (workers=%d), "
                     "dominance-excess column sweep vectorised over wavenumbers (numpy), "
                     "mean column by prefix sums; best of 2 full solves" % workers}
    if p_gpu64 is not None:
        out["rel_max_vs_fp64_gpu"] = float(np.abs(p - p_gpu64).max() / np.abs(p_gpu64).max())
    return out


_ORACLE_1CORE = r"""
import json, sys, time
sys.path.insert(0, %r)
import numpy as np
import oracle
from paper_2010_14132_amd import workloads as wl
out = {}
for name, prob in (("uniform_32x32x16", wl.uniform_white(seed=0)), ("plain_256x256x64", wl.plain_256())):
    g = prob.grid
    b = prob.rhs_exact()
    oracle.solve(b, g.dx, g.dy, g.dz, g.rho)
    t0 = time.perf_counter()
    oracle.solve(b, g.dx, g.dy, g.dz, g.rho)
    t = time.perf_counter() - t0
    out[name] = {"s_per_solve": t, "solves_per_s": 1.0 / t, "mpts_per_s": g.points / t / 1e6}
out["threads"] = oracle.num_threads()
print(json.dumps(out))
"""


def oracle_small_configs():
    """The oracle on the 32^2 x 16 and 256^2 x 64 workloads, on one core (a
    child process with OMP_NUM_THREADS=1, which touches no GPU) and on every
    core (this process)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", _ORACLE_1CORE % ROOT], env=env,
                       capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr[-400:]}
    one = json.loads(r.stdout.strip().splitlines()[-1])
    env["OMP_NUM_THREADS"] = str(os.cpu_count() or 1)
    r = subprocess.run([sys.executable, "-c", _ORACLE_1CORE % ROOT], env=env,
                       capture_output=True, text=True, timeout=600)
    allc = json.loads(r.stdout.strip().splitlines()[-1]) if r.returncode == 0 else {}
    return {"kind": "oracle", "one_core": one, "all_cores": allc}


# ------------------------------------------------------------ other workloads
def rel_max(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def config_forms(prob, forms, steps, warmup):
    """Solves/s and Mpts/s of each precision form on one workload (autotuned
    plans), the per-solve time distribution, and each FP32 form's rel_max
    against the FP64 GPU solve of the same input (whole field; the FP64
    solve's own parity with the oracle is a test's business)."""
    import torch
    from paper_2010_14132_amd import Plan
    g = prob.grid
    b64 = prob.rhs_exact() if prob.dtype == "f32" else prob.rhs
    ref = None
    res = {}
    for form in sorted(forms, key=lambda f: f != "fp64"):
        plan = Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.rho, precision=form)
        plan.autotune(reps=5)
        dt = torch.float64 if form == "fp64" else torch.float32
        b = torch.from_numpy(b64).to("cuda", dt)
        out = torch.empty_like(b)
        ms = time_calls(lambda: plan.solve(b, out=out), steps, warmup)
        d = time_distribution(lambda: plan.solve(b, out=out), max(50, steps))
        r = {"ms_per_solve": ms, "solves_per_s": 1e3 / ms, "mpts_per_s": g.points / ms / 1e3,
             "median_ms": d["median_ms"], "min_ms": d["min_ms"], "mean_ms": d["mean_ms"],
             "reps": d["reps"]}
        if form == "fp64":
            ref = out.double().cpu().numpy()
        elif ref is not None:
            r["rel_max_vs_fp64_gpu"] = rel_max(out.double().cpu().numpy(), ref)
        res[form] = r
        plan.close()
    return res


def config_monc_layout(prob, steps, warmup):
    """The headline workload with its fields in MONC's z-fastest layout
    ([nx][ny][nz]): ps_solve_zyx (x passes between the field and a
    [kx][j][k] buffer, y passes between that buffer and the spectrum, so
    40 B/pt as the level-major solve) against the level-major solve
    preceded and followed by explicit layout copies (torch permute copies,
    what a caller would otherwise run), FP32 with the in-register
    refinement, autotuned; per-pass event times (8 B/pt each)."""
    import torch
    from paper_2010_14132_amd import Plan
    g = prob.grid
    plan = Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.rho, precision="fp32_r2")
    plan.autotune(reps=5)
    b = torch.from_numpy(prob.rhs_as("f32")).cuda()
    bz = b.permute(2, 1, 0).contiguous()
    pz = torch.empty_like(bz)
    p = torch.empty_like(b)
    zyx = time_calls(lambda: plan.solve_zyx(bz, out=pz), steps, warmup)

    def unfused():
        bb = bz.permute(2, 1, 0).contiguous()
        plan.solve(bb, out=p)
        pz.copy_(p.permute(2, 1, 0))

    unf = time_calls(unfused, steps, warmup)
    lm = time_calls(lambda: plan.solve(b, out=p), steps, warmup)
    plan.profile(True)
    for _ in range(steps):
        plan.solve_zyx(bz, out=pz)
    kern = plan.profile_report()
    plan.profile(False)
    N = g.points
    xk = {}
    for name in ("fwd_x", "fft_y_fwd", "fft_y_inv", "inv_x"):
        if name in kern:
            tot, n = kern[name]
            ms = tot / steps
            xk[name] = {"ms_per_solve": ms, "gbs": 8.0 * N / (ms * 1e-3) / 1e9}
    res = {"zyx_ms_per_solve": zyx, "solves_per_s": 1e3 / zyx, "mpts_per_s": N / zyx / 1e3,
           "whole_solve_hbm_frac": 40.0 * N / (zyx * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "level_major_ms": lm, "level_major_with_two_transposes_ms": unf,
           "speedup_vs_transposes": unf / zyx, "zyx_kc": plan.info()["zyx_kc"],
           "passes": xk}
    plan.close()
    return res


def config_projection(prob, steps, warmup):
    """One projection step of the dynamical core on the headline grid
    (ps_project: divergence inside the forward x pass, solve, gradient
    correction), FP32 + in-register refinement and FP32 + physical-residual
    refinement, autotuned; velocities drawn N(0,1) by a seeded GPU generator.
    Beside it the plain solve on the same plan; per-kernel rates of the
    fused forward pass (reads u, v, w and writes the spectrum: 4 e bytes per
    point) and of the correction (reads p, u, v, w, writes u, v, w: 7 e)."""
    import torch
    from paper_2010_14132_amd import Plan
    g = prob.grid
    N = g.points
    gen = torch.Generator(device="cuda").manual_seed(5)
    res = {}
    for form in ("fp32_r2", "fp32_r1"):
        plan = Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.rho, precision=form)
        plan.autotune(reps=5)
        u, v, w = (torch.randn((g.nz, g.ny, g.nx), generator=gen, device="cuda")
                   for _ in range(3))
        p = torch.empty_like(u)
        b = torch.from_numpy(prob.rhs_as("f32")).cuda()
        # repeated projections of the same (already corrected) flow: the
        # work per step does not depend on the values
        proj = time_calls(lambda: plan.project(u, v, w, 10.0, out=p, correct=True), steps, warmup)
        solve = time_calls(lambda: plan.solve(b, out=p), steps, warmup)
        plan.profile(True)
        for _ in range(steps):
            plan.project(u, v, w, 10.0, out=p, correct=True)
        kern = plan.profile_report()
        plan.profile(False)
        kt = {}
        for name, bpp in (("fwd_x_divergence", 16.0), ("grad_correct", 28.0)):
            if name in kern:
                ms = kern[name][0] / steps
                kt[name] = {"ms_per_step": ms, "alg_bytes_per_point": bpp,
                            "gbs": bpp * N / (ms * 1e-3) / 1e9}
        res[form] = {"projection_ms": proj, "steps_per_s": 1e3 / proj,
                     "mpts_per_s": N / proj / 1e3, "plain_solve_ms": solve, "kernels": kt}
        plan.close()
        del u, v, w, p, b
    return res


def config_cg(prob):
    """The paper's Tables 1 and 2 on this hardware: the matrix-free Krylov
    solvers (CG on -D A, BiCGStab on A; Jacobi and no preconditioner, FP64)
    terminated at relative residuals 1e-2 ... 1e-8, iterations, time per
    solve (host clock around the call, which reads the convergence flag every
    16 iterations) and the mean difference from the FP64 direct solve,
    relative to the direct solution's mean magnitude; the direct solve's time
    beside it.  Algorithmic bytes per iteration: CG 88 B/pt (operator 16,
    update 48, direction 24), BiCGStab 168 B/pt (direction 32, two operator
    applications 24 + 16, two updates 48 + 48)."""
    import torch
    from paper_2010_14132_amd import CGSolver, Plan
    g = prob.grid
    b = torch.from_numpy(prob.rhs).cuda()
    plan = Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.rho, precision="fp64")
    plan.autotune(reps=5)
    direct = plan.solve(b)
    d_ms = time_calls(lambda: plan.solve(b, out=direct), 50, 5)
    dmean = direct.abs().mean().item()
    res = {"direct_fp64_ms": d_ms, "ladder": []}
    per_point = {"cg": 88, "bicgstab": 168}
    for method in ("cg", "bicgstab"):
        for precond in ("jacobi", "none"):
            s = CGSolver(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.rho, precond=precond,
                         method=method)
            s.solve(b, rtol=1e-2)  # warm-up
            for rtol in (1e-2, 1e-4, 1e-6, 1e-8):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, it, rel = s.solve(b, rtol=rtol, max_iter=100000)
                ms = (time.perf_counter() - t0) * 1e3
                nbytes = per_point[method] * g.points
                res["ladder"].append({
                    "method": method, "precond": precond, "rtol": rtol, "iterations": it,
                    "ms": ms, "ms_per_iteration": ms / max(it, 1), "final_rel_res": rel,
                    "mean_diff_vs_direct": (x - direct).abs().mean().item() / dmean,
                    "max_diff_vs_direct":
                        (x - direct).abs().max().item() / direct.abs().max().item(),
                    "iteration_bytes": nbytes,
                    "iteration_gbs": nbytes * max(it, 1) / (ms * 1e-3) / 1e9})
            s.close()
    plan.close()
    return res


def config_differentiation(steps, warmup):
    """512^2 x 128 differentiation workload: forward solve, adjoint solve and
    density gradient (one differentiation step = all three), FP32 form with
    FP64 mean / near-singular columns, and the FP64 forward solve beside it."""
    import torch
    from paper_2010_14132_amd import Plan
    from paper_2010_14132_amd import workloads as wl
    prob = wl.differentiation_512()
    g = prob.grid
    res = {"workload": "512x512x128 stretched grid, smooth RHS (seed 3), loss weights seed 1003"}
    for form in ("fp32", "fp64"):
        plan = Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.rho, precision=form)
        plan.autotune(reps=5)
        dt = torch.float64 if form == "fp64" else torch.float32
        b = torch.from_numpy(prob.rhs_exact()).to("cuda", dt)
        w = torch.from_numpy(prob.extra["w"]).to("cuda", dt)
        p, lam = torch.empty_like(b), torch.empty_like(b)

        def step():
            plan.solve(b, out=p)
            plan.solve_adjoint(w, out=lam)
            plan.grad_coeffs(lam, p)

        fwd = time_calls(lambda: plan.solve(b, out=p), steps, warmup)
        adj = time_calls(lambda: plan.solve_adjoint(w, out=lam), steps, warmup)
        stp = time_calls(step, steps, warmup)
        res[form] = {"forward_ms": fwd, "solves_per_s": 1e3 / fwd,
                     "mpts_per_s": g.points / fwd / 1e3, "adjoint_ms": adj,
                     "differentiation_step_ms": stp, "steps_per_s": 1e3 / stp}
        plan.close()
    return res


def config_batch(steps, warmup):
    """The 48-problem uneven batch (FP32): autotuned (each plan's kernels and
    the lane count), latency = median device time of one batched solve
    (events on the caller's stream around the whole replay) over >= 50
    replays, aggregate Mpts/s = total points / latency; beside it the same
    48 solves issued one after another on one stream, and the largest
    difference between a batched result and the same problem's standalone
    solve (zero: the same kernels on the same data)."""
    import torch
    from paper_2010_14132_amd import BatchPlan, Plan
    from paper_2010_14132_amd import workloads as wl
    probs = wl.batch_problems()
    npts = sum(p.grid.points for p in probs)
    batch = BatchPlan([p.grid for p in probs], precision="fp32")
    rhs = [torch.from_numpy(p.rhs_as("f32")).cuda() for p in probs]
    out = [torch.empty_like(r) for r in rhs]
    batch.autotune(rhs, out, reps=3)
    ms = time_calls(lambda: batch.solve(rhs, out), steps, warmup)
    d = time_distribution(lambda: batch.solve(rhs, out), max(50, steps))
    alg = sum(40.0 * p.grid.points for p in probs)  # five passes of 2 e bytes per point, e = 4
    res = {"workload": "48 problems, nx = ny in {64..512}, nz in {32..128}, stretch U[1, 1.05], "
                       "seed 4; problem i smooth RHS seed 4000+i",
           "problems": len(probs), "points": npts, "lanes": batch.info()["lanes"],
           "fp64_in_order": batch.info()["fp64_in_order"],
           "latency_median_ms": d["median_ms"], "latency_min_ms": d["min_ms"],
           "latency_mean_ms": d["mean_ms"], "reps": d["reps"], "ms_per_batch_mean": ms,
           "aggregate_mpts_per_s": npts / d["median_ms"] / 1e3,
           "batches_per_s": 1e3 / d["median_ms"],
           "alg_bytes": alg, "hbm_frac": alg / (d["median_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
    plans = []
    for p in probs:
        q = Plan(p.grid.nx, p.grid.ny, p.grid.nz, p.grid.dx, p.grid.dy, p.grid.dz, p.grid.rho,
                 precision="fp32")
        q.autotune(reps=3)  # the tune cache: the batch's own choices
        plans.append(q)
    seq = [torch.empty_like(r) for r in rhs]

    def sequential():
        for q, r, o in zip(plans, rhs, seq):
            q.solve(r, out=o)

    ds = time_distribution(sequential, max(20, steps // 2))
    torch.cuda.synchronize()
    res["max_abs_diff_vs_standalone"] = max((o - q).abs().max().item() for o, q in zip(out, seq))
    res["sequential_one_stream_median_ms"] = ds["median_ms"]
    res["speedup_vs_sequential"] = ds["median_ms"] / d["median_ms"]
    for q in plans:
        q.close()
    batch.close()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="fp32_r2", choices=["fp32", "fp32_r2", "fp32_r1", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="time only the headline form")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the planner's kernel choice instead of timing the variants")
    ap.add_argument("--tune-cache", default=None,
                    help="tune-cache file: loaded first if it exists, written after tuning "
                         "(so that profiled runs use the same kernels)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for scaling HBM counters)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other workloads (32^2x16, 256^2x64, 512^2x128, the batch)")
    ap.add_argument("--no-fast-cpu", action="store_true",
                    help="skip the fast CPU reference and the small-workload oracle timings")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(a sharded solve is a design only); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2010_14132_amd import Plan, binding
    from paper_2010_14132_amd import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    copy_gbs = None
    if args.tune_cache and os.path.exists(args.tune_cache):
        binding.tune_cache_load(args.tune_cache)
        print("bench: loaded tune cache %s" % args.tune_cache, file=sys.stderr, flush=True)
    if args.copy_calibration:
        # a plain copy of known size: 1 GiB read + 1 GiB written per launch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        copy_gbs = 2 * src.numel() * 4 / (e0.elapsed_time(e1) / 5 * 1e-3) / 1e9
        print("bench: 1 GiB device copy %.0f GB/s" % copy_gbs, file=sys.stderr, flush=True)
        del src, dst
    prob = wl.precision_1024("f32")
    g = prob.grid
    N = g.points
    print("bench: generated %s (%d points)" % (prob.name, N), file=sys.stderr, flush=True)
    b32 = torch.from_numpy(prob.rhs_as("f32")).cuda()
    b64 = torch.from_numpy(prob.rhs_exact()).cuda()  # the same FP32 values, promoted

    forms = [args.precision] if args.no_variants else \
        [args.precision] + [f for f in ("fp64", "fp32", "fp32_r2", "fp32_r1") if f != args.precision]
    results = {}
    outputs = {}
    for form in forms:
        plan = Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.rho, precision=form)
        if not args.no_autotune:
            plan.autotune(reps=5)
        b = b64 if form == "fp64" else b32
        out = torch.empty_like(b)
        steps = args.steps if form == args.precision else max(5, args.steps // 2)
        ms = time_solves(plan, b, out, steps, args.warmup)
        results[form] = {"ms_per_solve": ms, "solves_per_s": 1e3 / ms, "mpts_per_s": N / ms / 1e3,
                         "fp64_columns": plan.info()["fp64_columns"], "steps": steps,
                         "kernels": {k: plan.info()[k] for k in
                                     ("fft_variant_x", "fft_variant_xi", "fft_variant_y",
                                      "column_variant", "chunks", "special_variant", "fp64_beside",
                                      "xy_chunks")}}
        outputs[form] = out
        dist = time_distribution(lambda: plan.solve(b, out=out), max(50, steps))
        results[form].update({"median_ms": dist["median_ms"], "min_ms": dist["min_ms"],
                              "mean_ms": dist["mean_ms"], "reps": dist["reps"]})
        print("bench: %-8s %.4f ms/solve (median %.4f over %d)"
              % (form, ms, dist["median_ms"], dist["reps"]), file=sys.stderr, flush=True)
        if form == args.precision:
            # the differentiation path of the same form: the adjoint solve
            # (gp = the right-hand side) and the density gradient from the
            # adjoint field and the solution
            lam = torch.empty_like(b)
            results[form]["adjoint_ms_per_solve"] = time_calls(
                lambda: plan.solve_adjoint(b, out=lam), steps, args.warmup)
            results[form]["grad_rho_ms"] = time_calls(
                lambda: plan.grad_coeffs(lam, out), steps, args.warmup)
            print("bench: %-8s adjoint %.4f ms, grad-rho %.4f ms"
                  % (form, results[form]["adjoint_ms_per_solve"], results[form]["grad_rho_ms"]),
                  file=sys.stderr, flush=True)
        # per-kernel event timing (a separate pass: events add a little per launch)
        plan.profile(True)
        for _ in range(steps):
            plan.solve(b, out=out)
        kern = plan.profile_report()
        plan.profile(False)
        e = 8 if form == "fp64" else 4
        info = plan.info()
        # the refinement repeats the y, column and backward x passes under
        # the same kernel names (its second x forward is fwd_x_residual)
        r1 = form == "fp32_r1"
        results[form]["chunks"] = info["chunks"]
        kt = {}
        for name, (tot, n) in kern.items():
            avg = tot / n
            per_solve_ms = tot / steps
            if r1 and name == "inv_x":
                # one plain pass and one accumulating pass
                alg = (kernel_bytes_per_point(name, e, g.nx)
                       + kernel_bytes_per_point(name, e, g.nx, accumulate=True)) * N
            else:
                npass = 2 if (r1 and name in ("fft_y_fwd", "columns", "fft_y_inv")) else 1
                alg = kernel_bytes_per_point(name, e, g.nx) * N * npass  # per solve
            bpp = alg / N
            kt[name] = {"avg_ms": avg, "launches_per_solve": n / steps, "ms_per_solve": per_solve_ms,
                        "alg_bytes_per_solve": alg,
                        "gbs": (alg / (per_solve_ms * 1e-3) / 1e9) if bpp else None}
        results[form]["kernel_times"] = kt
        # the whole solve against HBM peak: the algorithmic bytes of all its
        # passes over the solve's wall time (streams overlapped)
        alg_total = sum(v["alg_bytes_per_solve"] for v in kt.values())
        results[form]["whole_solve"] = {
            "alg_bytes": alg_total, "bytes_per_point": alg_total / N,
            "gbs": alg_total / (results[form]["ms_per_solve"] * 1e-3) / 1e9,
            "hbm_frac": alg_total / (results[form]["ms_per_solve"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
        if form == args.precision:
            kernels = kt
        plan.close()
    if args.tune_cache:
        binding.tune_cache_save(args.tune_cache)
    # dominant kernel: the largest share of the solve among the kernels that
    # run as one launch per solve (one launch = one full pass over the data;
    # passes taken in level or kx ranges launch in pieces)
    single = {k: v for k, v in kernels.items()
              if v["gbs"] and abs(v["launches_per_solve"] - 1.0) < 1e-9
              and not k.startswith("fft_y")}
    dom = max(single, key=lambda k: kernels[k]["ms_per_solve"])
    dk = kernels[dom]
    achieved = dk["gbs"] or 0.0

    # accuracy: against the FP64 GPU solve (full field; parity of every form
    # with the oracle at this size is checked by the GPU tests)
    errs = {}
    if "fp64" in outputs:
        ref = outputs["fp64"].double()
        den = ref.abs().max().item()
        for form, o in outputs.items():
            if form != "fp64":
                d = o.double() - ref
                errs[form + "_vs_fp64_gpu_rel_max"] = d.abs().max().item() / den
                errs[form + "_vs_fp64_gpu_rel_l2"] = (d.norm() / ref.norm()).item()

    line = {
        "metric": "Poisson solves/s & Mpts/s, 1024^2x128 fp32+refine vs fp64; % of HBM peak",
        "value": results[args.precision]["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": results[args.precision]["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": "1024x1024x128 stretched grid (dz=20m*1.03^k), rho=exp(-z/8km), "
                               "smooth k^-2 RHS + 1% noise, seed 2",
                   "nx": g.nx, "ny": g.ny, "nz": g.nz, "precision": args.precision,
                   "global_batch": 1, "parallelism": "none (1 GPU)"},
        "mpts_per_s": results[args.precision]["mpts_per_s"],
        "forms": results,
        "errors": errs,
        "kernels": kernels,
        # achieved: algorithmic bytes of the dominant kernel per solve over its
        # event-timed duration per solve (profiled pass of `steps` solves);
        # traffic: measured HBM bytes per solve of that kernel
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.precision, dom),
                     "algorithmic_bytes": dk["alg_bytes_per_solve"]},
    }
    if copy_gbs is not None:
        line["device_copy_gbs"] = copy_gbs
    if "fp64" in results and args.precision != "fp64":
        line["speedup_vs_fp64"] = results["fp64"]["ms_per_solve"] / results[args.precision]["ms_per_solve"]
    if not args.no_configs:
        print("bench: MONC layout", file=sys.stderr, flush=True)
        line["monc_layout"] = config_monc_layout(prob, args.steps, args.warmup)
        print("bench: projection step", file=sys.stderr, flush=True)
        line["projection_step"] = config_projection(prob, args.steps, args.warmup)
    line["whole_solve_hbm"] = results[args.precision]["whole_solve"]
    line["timing"] = {k: results[args.precision][k] for k in ("median_ms", "min_ms", "mean_ms",
                                                               "reps")}
    if not args.no_fast_cpu:
        print("bench: fast CPU reference (FP64 scipy FFT + vectorised sweep)", file=sys.stderr,
              flush=True)
        p64 = outputs["fp64"].cpu().numpy() if "fp64" in outputs else None
        line["fast_cpu_reference"] = fast_cpu_reference(prob, p64)
        del p64
    del outputs
    if not args.no_configs:
        from paper_2010_14132_amd import workloads as wl2
        configs = {}
        print("bench: 32x32x16 plain", file=sys.stderr, flush=True)
        configs["uniform_32x32x16"] = {
            "workload": "32x32x16, dz = 40 m, rho = 1, white RHS (seed 0)",
            "forms": config_forms(wl2.uniform_white(seed=0), ["fp64", "fp32_r2"],
                                  max(200, args.steps), args.warmup)}
        print("bench: 256x256x64 plain", file=sys.stderr, flush=True)
        configs["plain_256x256x64"] = {
            "workload": "256x256x64 stretched grid, rho(z), smooth RHS (seed 1)",
            "forms": config_forms(wl2.plain_256(), ["fp64", "fp32", "fp32_r2", "fp32_r1"],
                                  max(100, args.steps), args.warmup)}
        print("bench: 256x256x64 matrix-free CG ladder", file=sys.stderr, flush=True)
        configs["plain_256x256x64"]["cg_table1"] = config_cg(wl2.plain_256())
        print("bench: 512x512x128 differentiation", file=sys.stderr, flush=True)
        configs["differentiation_512x512x128"] = config_differentiation(args.steps, args.warmup)
        print("bench: 48-problem uneven batch", file=sys.stderr, flush=True)
        configs["batch_48"] = config_batch(args.steps, args.warmup)
        line["configs"] = configs
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(g, g.nz)
        if not args.no_fast_cpu:
            line["cpu_baseline"]["small_workloads"] = oracle_small_configs()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
