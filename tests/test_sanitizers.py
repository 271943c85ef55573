"""Host-side sanitizer runs (CPU only): the oracle built with gcc's
AddressSanitizer and UndefinedBehaviorSanitizer under its pins, and the
library's host code built with clang's (device code unchanged) under the
host-side ABI tests, each in a subprocess with the matching runtime
preloaded.  A memory error or undefined behaviour aborts the subprocess."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.slow


def _run(env_extra, tests):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", **env_extra)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-m", "not gpu",
                        "-p", "no:cacheprovider"] + tests, cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=1200)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout


def test_oracle_under_asan_ubsan():
    import oracle
    oracle.build(sanitize=True)
    libs = [subprocess.check_output(["gcc", "-print-file-name=" + n], text=True).strip()
            for n in ("libasan.so", "libubsan.so")]
    _run({"LD_PRELOAD": ":".join(libs), "PS_ORACLE_SANITIZE": "1"},
         ["tests/test_oracle_pins.py", "tests/test_golden.py", "tests/test_cg_reference.py"])


def test_host_library_under_asan_ubsan():
    from paper_2010_14132_amd import build as b
    srcs = glob.glob(os.path.join(b.CSRC, "*"))
    if not os.path.exists(b.LIB_ASAN) or \
            os.path.getmtime(b.LIB_ASAN) < max(os.path.getmtime(f) for f in srcs):
        b.build(verbose=False, sanitize=True)
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("clang ASan runtime not found")
    _run({"LD_PRELOAD": rt[-1], "PS_LIBRARY": b.LIB_ASAN}, ["tests/test_abi_host.py"])
