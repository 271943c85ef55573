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
roofline of the dominant kernel, and the CPU oracle timed on a bounded sample.
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


def sampled_oracle_error(p: np.ndarray, b: np.ndarray, g, modes) -> float:
    """Relative error of sampled wavenumber columns against the oracle's
    column solve of a plain DFT of the input (test infrastructure)."""
    import oracle
    nz, ny, nx = p.shape
    scale, err = 0.0, 0.0
    for kx, ky in modes:
        ex = np.exp(-2j * np.pi * kx * np.arange(nx) / nx)
        ey = np.exp(-2j * np.pi * ky * np.arange(ny) / ny)
        s = 4 * np.sin(np.pi * kx / nx) ** 2 / g.dx ** 2 + 4 * np.sin(np.pi * ky / ny) ** 2 / g.dy ** 2
        want = oracle.column_solve(s, (b @ ex) @ ey, g.dz, g.rho)
        got = (p @ ex) @ ey
        scale = max(scale, np.abs(want).max())
        err = max(err, np.abs(got - want).max())
    return err / scale


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
            "mpts_per_s": g.nx * g.ny * nz_full / t_full / 1e6}


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


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="fp32_r2", choices=["fp32", "fp32_r2", "fp32_r1", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="time only the headline form")
    ap.add_argument("--no-oracle-check", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the planner's kernel choice instead of timing the variants")
    ap.add_argument("--tune-cache", default=None,
                    help="tune-cache file: loaded first if it exists, written after tuning "
                         "(so that profiled runs use the same kernels)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for scaling HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(the sharded design is described in DESIGN.md); use --gpus 1", file=sys.stderr)
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
                                      "column_variant", "chunks")}}
        outputs[form] = out
        print("bench: %-8s %.4f ms/solve" % (form, ms), file=sys.stderr, flush=True)
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
        if form == args.precision:
            kernels = kt
        plan.close()
    if args.tune_cache:
        binding.tune_cache_save(args.tune_cache)
    # dominant kernel: the largest share of the solve among the kernels that
    # run once per transform pass (one launch = one full pass over the data)
    single = {k: v for k, v in kernels.items()
              if v["gbs"] and abs(v["launches_per_solve"] - round(v["launches_per_solve"])) < 1e-9
              and not k.startswith("fft_y")}
    dom = max(single, key=lambda k: kernels[k]["ms_per_solve"])
    dk = kernels[dom]
    achieved = dk["gbs"] or 0.0

    # accuracy: against the FP64 GPU solve (full field) and the oracle (sampled)
    errs = {}
    if "fp64" in outputs:
        ref = outputs["fp64"].double()
        den = ref.abs().max().item()
        for form, o in outputs.items():
            if form != "fp64":
                errs[form + "_vs_fp64_gpu_rel_max"] = (o.double() - ref).abs().max().item() / den
    if not args.no_oracle_check:
        modes = [(1, 0), (0, 1), (1, 1), (3, 7), (100, 200), (512, 512), (0, 511)]
        p_head = outputs[args.precision].double().cpu().numpy()
        errs["headline_vs_oracle_sampled_rel"] = sampled_oracle_error(
            p_head, prob.rhs_exact(), g, modes)

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
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(g, g.nz)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
