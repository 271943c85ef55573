"""Differentiation form: p = S(b; rho) through the torch.autograd.Function
of the binding (forward solve, adjoint solve, density-gradient kernel), with
loss L = sum(w * p).

* 512^2 x 128 stretched grid (seed 3, loss weights w seed 1003), gradients
  of the FP32 form (FP64 mean / near-singular columns) and of the FP64 form
  against central finite differences in FP64 (step 1e-3) along 32 seeded
  unit directions (seed 2003): 16 in b, and 16 in rho applied as
  rho_k (1 + h d_k) so the densities stay positive.
* A separate 16 x 16 x 8 problem of the same recipe (seed 3003) against the
  dense bordered system: grad_b = K^-T w by LAPACK, grad_rho by complex-step
  differentiation of the dense assembly.
"""
import numpy as np
import pytest

from paper_2010_14132_amd import workloads as wl
from tests import dense_check as dc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

H = 1e-3
NDIR = 16


def announce(msg):
    print("\n[gpu] " + msg, flush=True)


def make_plan(g, precision):
    from paper_2010_14132_amd import Plan
    return Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.rho, precision=precision)


def autograd_grads(g, b_np, w_np, precision):
    """(grad_b, grad_rho, L) from one forward + backward through the
    autograd function."""
    from paper_2010_14132_amd import poisson_solve
    dt = torch.float64 if precision == "fp64" else torch.float32
    plan = make_plan(g, precision)
    b = torch.from_numpy(b_np).to("cuda", dt).requires_grad_(True)
    rho = torch.tensor(g.rho, dtype=torch.float64, requires_grad=True)
    w = torch.from_numpy(w_np).to("cuda", dt)
    p = poisson_solve(b, rho, plan)
    loss = (w.double() * p.double()).sum()
    loss.backward()
    torch.cuda.synchronize()
    out = (b.grad.double().cpu().numpy(), rho.grad.double().cpu().numpy(), float(loss))
    plan.close()
    return out


def test_c3_autograd_against_fd_512():
    prob = wl.differentiation_512()
    g = prob.grid
    b64 = prob.rhs_exact()          # the FP32-rounded draw, promoted
    w = prob.extra["w"].astype(np.float32).astype(np.float64)
    announce("C3 512^2x128: autograd fp32 + fp64")
    gb32, gr32, _ = autograd_grads(g, prob.rhs_as("f32"), w.astype(np.float32), "fp32")
    gb64, gr64, L0 = autograd_grads(g, b64, w, "fp64")

    # loss evaluations in FP64 on the GPU
    plan = make_plan(g, "fp64")
    wt = torch.from_numpy(w).cuda()
    bt = torch.from_numpy(b64).cuda()

    def loss(bb, rho=None):
        if rho is not None:
            plan.set_coeffs(rho)
        p = plan.solve(bb)
        return float((wt * p).sum())

    rng = np.random.default_rng(2003)
    worst = {"b32": 0.0, "b64": 0.0, "r32": 0.0, "r64": 0.0}
    announce("C3 FD along %d b-directions" % NDIR)
    nb32 = np.linalg.norm(gb32)
    nb64 = np.linalg.norm(gb64)
    for _ in range(NDIR):
        d = rng.standard_normal(g.shape)
        d /= np.linalg.norm(d)
        dt_ = torch.from_numpy(d).cuda()
        fd = (loss(bt + H * dt_) - loss(bt - H * dt_)) / (2 * H)
        worst["b64"] = max(worst["b64"], abs(np.vdot(gb64, d) - fd) / nb64)
        worst["b32"] = max(worst["b32"], abs(np.vdot(gb32, d) - fd) / nb32)
    announce("C3 FD along %d rho-directions" % NDIR)
    rho0 = g.rho.copy()
    n64 = np.linalg.norm(gr64 * rho0)
    n32 = np.linalg.norm(gr32 * rho0)
    for _ in range(NDIR):
        d = rng.standard_normal(g.nz)
        d /= np.linalg.norm(d)
        fd = (loss(bt, rho0 * (1 + H * d)) - loss(bt, rho0 * (1 - H * d))) / (2 * H)
        worst["r64"] = max(worst["r64"], abs(np.dot(gr64 * rho0, d) - fd) / n64)
        worst["r32"] = max(worst["r32"], abs(np.dot(gr32 * rho0, d) - fd) / n32)
    plan.set_coeffs(rho0)
    plan.close()
    print("C3 worst directional errors (relative to the gradient norm): %s" % worst)
    # b-directions: L is linear in b, so the difference quotient is exact up
    # to rounding; rho-directions carry the O(h^2) truncation of the central
    # difference.
    assert worst["b64"] < 1e-9
    assert worst["r64"] < 1e-5
    assert worst["b32"] < 1e-5
    assert worst["r32"] < 1e-4
    # Euler identity: V is unchanged by rho -> c rho, so sum_k rho_k g_k = 0
    assert abs(np.dot(rho0, gr64)) < 1e-9 * np.abs(rho0 * gr64).sum()


def complex_step_grad(b, w, g):
    """dL/drho_k of L = <w, S b> by complex-step differentiation of the dense
    bordered solve (no Fourier transform, no oracle)."""
    hc = 1e-30
    out = np.zeros(g.nz)
    rhs = np.append(b.ravel(), 0.0).astype(complex)
    for k in range(g.nz):
        rc = np.asarray(g.rho, dtype=complex).copy()
        rc[k] += 1j * hc
        A = dc.dense_operator(b.shape, g.dx, g.dy, g.dz, rc)
        sol = np.linalg.solve(dc.bordered(A), rhs)
        out[k] = np.vdot(w.ravel(), sol[:-1]).imag / hc
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c3_dense_transpose_16x16x8(precision):
    announce("C3 dense-transpose 16x16x8 %s" % precision)
    prob = wl.stretched_smooth(16, 16, 8, seed=3003, dtype="f32" if precision == "fp32" else "f64")
    g = prob.grid
    b = prob.rhs_exact()
    w = np.random.default_rng(3004).standard_normal(g.shape)
    if precision == "fp32":
        w = w.astype(np.float32).astype(np.float64)
    want_b = dc.dense_adjoint(w, g.dx, g.dy, g.dz, g.rho)
    want_r = complex_step_grad(b, w, g)
    dt = np.float64 if precision == "fp64" else np.float32
    gb, gr, _ = autograd_grads(g, b.astype(dt), w.astype(dt), precision)
    eb = np.abs(gb - want_b).max() / np.abs(want_b).max()
    er = np.abs(gr - want_r).max() / np.abs(want_r).max()
    print("grad_b rel %.3e, grad_rho rel %.3e" % (eb, er))
    tol = 1e-11 if precision == "fp64" else 1e-5
    assert eb < tol
    assert er < tol


def test_shared_plan_two_densities_one_backward():
    """Two forwards through one plan at different densities, one loss, one
    backward: each forward's gradient must use its own operator (the
    backward sets that forward's densities for the adjoint solve and the
    density gradient and restores the plan's current ones).  Checked
    against the dense bordered system and complex-step differentiation."""
    from paper_2010_14132_amd import poisson_solve
    announce("shared plan, two densities, one backward 16x16x8 fp64")
    prob = wl.stretched_smooth(16, 16, 8, seed=3005, dtype="f64")
    g = prob.grid
    b = prob.rhs_exact()
    rho1 = g.rho.copy()
    rho2 = g.rho * np.linspace(0.7, 1.4, g.nz)
    rng = np.random.default_rng(3006)
    w1, w2 = rng.standard_normal(g.shape), rng.standard_normal(g.shape)
    plan = make_plan(g, "fp64")
    bt = torch.from_numpy(b).cuda().requires_grad_(True)
    r1 = torch.tensor(rho1, dtype=torch.float64, requires_grad=True)
    r2 = torch.tensor(rho2, dtype=torch.float64, requires_grad=True)
    p1 = poisson_solve(bt, r1, plan)
    p2 = poisson_solve(bt, r2, plan)  # the plan now holds rho2
    loss = (torch.from_numpy(w1).cuda() * p1).sum() + (torch.from_numpy(w2).cuda() * p2).sum()
    loss.backward()
    torch.cuda.synchronize()
    want_b = (dc.dense_adjoint(w1, g.dx, g.dy, g.dz, rho1)
              + dc.dense_adjoint(w2, g.dx, g.dy, g.dz, rho2))
    g2 = wl.Grid(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, rho2)
    eb = np.abs(bt.grad.cpu().numpy() - want_b).max() / np.abs(want_b).max()
    e1 = np.abs(r1.grad.numpy() - complex_step_grad(b, w1, g)).max()
    e2 = np.abs(r2.grad.numpy() - complex_step_grad(b, w2, g2)).max()
    print("grad_b rel %.3e, grad_rho abs %.3e %.3e" % (eb, e1, e2))
    assert eb < 1e-11
    assert e1 < 1e-11 * np.abs(r1.grad.numpy()).max()
    assert e2 < 1e-11 * np.abs(r2.grad.numpy()).max()
    assert np.array_equal(plan.rho, rho2)  # the plan's own densities restored
    plan.close()
