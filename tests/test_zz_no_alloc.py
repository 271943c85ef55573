"""ps_grad_coeffs_noalloc (the density gradient with its partial sums in the
library's fixed device array, for callers that cannot allocate) against
ps_grad_coeffs, through the C ABI: two calls in a row, the second on a
smaller problem, each equal to the allocating entry point bit for bit (same
kernels, same fixed-order reduction), and the first also against the
oracle."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2010_14132_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _call(plan, lam, p, noalloc):
    from paper_2010_14132_amd import binding
    lib = binding.load()
    g = torch.empty(plan.nz, dtype=torch.float64, device="cuda")
    plan._sync_stream()
    fn = lib.ps_grad_coeffs_noalloc if noalloc else lib.ps_grad_coeffs
    rc = fn(plan._h, ctypes.c_void_p(lam.data_ptr()), ctypes.c_void_p(p.data_ptr()),
            ctypes.c_void_p(g.data_ptr()))
    binding.check(rc, "grad")
    return g


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_grad_coeffs_noalloc_matches_allocating_entry_point(precision):
    from paper_2010_14132_amd import Plan
    print("\n[gpu] grad_coeffs_noalloc %s" % precision, flush=True)
    dt = torch.float64 if precision == "fp64" else torch.float32
    # first a problem with many blocks and levels, then a smaller one: the
    # second call must not see the first call's partials
    for n, nz, seed in ((512, 128, 41), (48, 9, 42)):
        g = wl.stretched_grid(n, n, nz)
        rng = np.random.default_rng(seed)
        lam = torch.from_numpy(rng.standard_normal(g.shape)).to("cuda", dt)
        p = torch.from_numpy(rng.standard_normal(g.shape) + 0.5).to("cuda", dt)
        plan = Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.rho, precision=precision)
        got = _call(plan, lam, p, noalloc=True)
        want = _call(plan, lam, p, noalloc=False)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (n, nz)
        if n == 48:
            ref = oracle.grad_rho(lam.double().cpu().numpy(), p.double().cpu().numpy(),
                                  g.dx, g.dy, g.dz, g.rho)
            err = np.abs(got.cpu().numpy() - ref).max() / np.abs(ref).max()
            assert err < 1e-12, err
        plan.close()
