"""Build the HIP library libpressure_solve.so for gfx950 with hipcc.

Every source under csrc/ is compiled (in parallel) to an object under
_build/ and linked into paper_2010_14132_amd/libpressure_solve.so.  The build
always recompiles; it runs on a machine without a GPU (hipcc cross-compiles).

build(sanitize=True) builds a CPU-checking variant instead,
_build_asan/libpressure_solve_asan.so: the host code instrumented with
AddressSanitizer and UndefinedBehaviorSanitizer (device code unchanged), for
running the host-side tests with the clang ASan runtime preloaded.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpressure_solve.so")
ARCH = os.environ.get("PS_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    "-mcode-object-version=5",
    # packed FP32 instructions are disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
]


BUILD_ASAN = os.path.join(HERE, "_build_asan")
LIB_ASAN = os.path.join(BUILD_ASAN, "libpressure_solve_asan.so")
# host-side sanitizers only: each -fsanitize applies to the host compilation
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all",
             "-g"]


def _compile(src: str, sanitize: bool = False) -> str:
    obj = os.path.join(BUILD_ASAN if sanitize else BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + (SAN_FLAGS if sanitize else []) + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if warn:
        sys.stderr.write(warn + "\n")
    return obj


def build(verbose: bool = True, sanitize: bool = False) -> str:
    out_dir = BUILD_ASAN if sanitize else BUILD
    lib = LIB_ASAN if sanitize else LIB
    os.makedirs(out_dir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")), 8)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, sanitize), srcs))
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    if sanitize:
        cmd += ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-shared-libsan"]
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    build()
