"""Thin ctypes binding of libpressure_solve.so (the C ABI in
include/pressure_solve.h).  Argument marshalling only: every step of the
solve runs in the library's HIP kernels.  PyTorch supplies device memory and
the current stream.

The library is loaded on first use; if it has not been built, or a call is
made without a GPU, an error is raised -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PS_LIBRARY selects another build of the same library (the host-sanitizer
# build of the CPU tests); by default the in-tree build.
LIB_PATH = os.environ.get("PS_LIBRARY") or os.path.join(_HERE, "libpressure_solve.so")

PS_FP64, PS_FP32, PS_FP32_R2, PS_FP32_R1 = 0, 1, 2, 3
PRECISIONS = {"fp64": PS_FP64, "fp32": PS_FP32, "fp32_r2": PS_FP32_R2, "fp32_r1": PS_FP32_R1}
STATUS = {0: "PS_OK", 1: "PS_EINVAL", 2: "PS_EUNSUPPORTED", 3: "PS_ENOMEM", 4: "PS_EHIP",
          5: "PS_ESTATE"}

_lib = None
_lock = threading.Lock()
_vp = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


class PlanInfo(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("precision", ctypes.c_int), ("fp64_columns", ctypes.c_int),
                ("tau", ctypes.c_double), ("fft_variant_x", ctypes.c_int),
                ("fft_variant_y", ctypes.c_int), ("spectrum_elems", ctypes.c_size_t),
                ("column_variant", ctypes.c_int), ("chunks", ctypes.c_int),
                ("fft_variant_xi", ctypes.c_int), ("special_variant", ctypes.c_int),
                ("zyx_kc", ctypes.c_int), ("fp64_beside", ctypes.c_int),
                ("xy_chunks", ctypes.c_int)]


# name -> (restype, argtypes); mirrors include/pressure_solve.h
SIGNATURES = {
    "ps_plan_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_double, ctypes.c_double, _D, _D, ctypes.c_int,
                                      ctypes.c_double, _vp]),
    "ps_plan_destroy": (ctypes.c_int, [_vp]),
    "ps_plan_set_stream": (ctypes.c_int, [_vp, _vp]),
    "ps_plan_set_coeffs": (ctypes.c_int, [_vp, _D]),
    "ps_solve": (ctypes.c_int, [_vp, _vp, _vp]),
    "ps_solve_adjoint": (ctypes.c_int, [_vp, _vp, _vp]),
    "ps_solve_zyx": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int]),
    "ps_project": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_double, _vp, ctypes.c_int]),
    "ps_grad_coeffs": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "ps_grad_coeffs_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "ps_workspace_bytes": (ctypes.c_size_t, [_vp]),
    "ps_plan_query": (ctypes.c_int, [_vp, ctypes.POINTER(PlanInfo)]),
    "ps_plan_autotune": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ps_tune_cache_save": (ctypes.c_int, [ctypes.c_char_p]),
    "ps_tune_cache_load": (ctypes.c_int, [ctypes.c_char_p]),
    "ps_forward_transform": (ctypes.c_int, [_vp, _vp, _vp]),
    "ps_spectral_solve": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    "ps_inverse_transform": (ctypes.c_int, [_vp, _vp, _vp]),
    "ps_batch_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, _I, _I, _I, _D, _D,
                                       ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.c_int, _vp]),
    "ps_batch_solve": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp)]),
    "ps_batch_destroy": (ctypes.c_int, [_vp]),
    "ps_batch_set_stream": (ctypes.c_int, [_vp, _vp]),
    "ps_batch_autotune": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_int]),
    "ps_batch_query": (ctypes.c_int, [_vp, _I, _I, _I]),
    "ps_batch_set_fp64_order": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ps_batch_status": (ctypes.c_int, [_vp]),
    "ps_batch_set_mode": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ps_batch_set_lanes": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ps_plan_profile": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ps_plan_profile_report": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_char_p),
                                              ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_int)]),
    "ps_cg_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_double, ctypes.c_double, _D, _D, ctypes.c_int, _vp]),
    "ps_cg_solve": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int, _I,
                                   ctypes.POINTER(ctypes.c_double)]),
    "ps_cg_set_stream": (ctypes.c_int, [_vp, _vp]),
    "ps_cg_set_method": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ps_cg_workspace_bytes": (ctypes.c_size_t, [_vp]),
    "ps_cg_destroy": (ctypes.c_int, [_vp]),
    "ps_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "ps_last_error": (ctypes.c_char_p, []),
}


class PressureSolveError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str = ""):
        self.status = status
        super().__init__("%s failed: %s%s" % (what, STATUS.get(status, str(status)),
                                               (" (%s)" % detail) if detail else ""))


def load():
    """Load the HIP library (after torch, so both use one HIP runtime)."""
    global _lib
    with _lock:
        if _lib is None:
            import torch  # noqa: F401  -- loads the HIP runtime the library binds to
            if not os.path.exists(LIB_PATH):
                raise RuntimeError("libpressure_solve.so is not built (%s); run "
                                   "paper_2010_14132_amd.build.build()" % LIB_PATH)
            lib = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def check(status: int, what: str):
    if status != 0:
        detail = load().ps_last_error()
        raise PressureSolveError(status, what, detail.decode() if detail else "")


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _stream_handle():
    import torch
    return _vp(torch.cuda.current_stream().cuda_stream)


class Plan:
    """A planned solve for one grid and precision (the C ABI's ps_plan).

    precision: "fp64", "fp32" (FP64 mean and near-singular columns),
    "fp32_r2" (plus in-register refinement of each column solve) or
    "fp32_r1" (plus one step of iterative refinement on the 3D residual).
    """

    def __init__(self, nx, ny, nz, dx, dy, dz, rho, precision="fp64", tau=0.0, device=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the pressure-solve library needs a GPU (no CPU fallback)")
        lib = load()
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.dx, self.dy = float(dx), float(dy)
        self.dz = np.ascontiguousarray(dz, dtype=np.float64)
        self.rho = np.ascontiguousarray(rho, dtype=np.float64)
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        h = _vp()
        with torch.cuda.device(self.device):
            check(lib.ps_plan_create(ctypes.byref(h), self.nx, self.ny, self.nz, self.dx, self.dy,
                                     _dptr(self.dz), _dptr(self.rho), PRECISIONS[precision],
                                     float(tau), _stream_handle()), "ps_plan_create")
        self._h = h

    # -- helpers
    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def _sync_stream(self):
        check(load().ps_plan_set_stream(self._h, _stream_handle()), "ps_plan_set_stream")

    def _check_field(self, t, name):
        import torch
        if not isinstance(t, torch.Tensor):
            raise TypeError("%s must be a torch tensor" % name)
        if t.device != self.device or t.dtype != self.dtype or tuple(t.shape) != self.shape \
                or not t.is_contiguous():
            raise ValueError("%s must be a contiguous %s tensor of shape %s on %s (got %s %s %s)"
                             % (name, self.dtype, self.shape, self.device, t.dtype,
                                tuple(t.shape), t.device))

    def _out(self, out):
        import torch
        if out is None:
            return torch.empty(self.shape, dtype=self.dtype, device=self.device)
        self._check_field(out, "out")
        return out

    # -- the C ABI
    def solve(self, rhs, out=None):
        self._check_field(rhs, "rhs")
        out = self._out(out)
        self._sync_stream()
        check(load().ps_solve(self._h, _vp(rhs.data_ptr()), _vp(out.data_ptr())), "ps_solve")
        return out

    def solve_adjoint(self, gp, out=None):
        self._check_field(gp, "gp")
        out = self._out(out)
        self._sync_stream()
        check(load().ps_solve_adjoint(self._h, _vp(gp.data_ptr()), _vp(out.data_ptr())),
              "ps_solve_adjoint")
        return out

    @property
    def shape_zyx(self):
        """MONC's p%data(z,y,x) as a C array: [nx][ny][nz], z fastest."""
        return (self.nx, self.ny, self.nz)

    def solve_zyx(self, rhs, out=None, adjoint=False):
        """ps_solve / ps_solve_adjoint for fields in MONC's z-fastest layout
        (tensors of shape [nx][ny][nz])."""
        import torch
        for t, nm in ((rhs, "rhs"),) + (((out, "out"),) if out is not None else ()):
            if t.device != self.device or t.dtype != self.dtype \
                    or tuple(t.shape) != self.shape_zyx or not t.is_contiguous():
                raise ValueError("%s must be a contiguous %s tensor of shape %s on %s"
                                 % (nm, self.dtype, self.shape_zyx, self.device))
        if out is None:
            out = torch.empty(self.shape_zyx, dtype=self.dtype, device=self.device)
        self._sync_stream()
        check(load().ps_solve_zyx(self._h, _vp(rhs.data_ptr()), _vp(out.data_ptr()),
                                  int(bool(adjoint))), "ps_solve_zyx")
        return out

    def project(self, u, v, w, dt, out=None, correct=True):
        """One projection step: p = S(div(u, v, w)/dt) with the divergence
        formed in the forward pass; with correct, (u, v, w) -= dt G p in
        place.  Returns p."""
        for t, nm in ((u, "u"), (v, "v"), (w, "w")):
            self._check_field(t, nm)
        out = self._out(out)
        self._sync_stream()
        check(load().ps_project(self._h, _vp(u.data_ptr()), _vp(v.data_ptr()),
                                _vp(w.data_ptr()), float(dt), _vp(out.data_ptr()),
                                int(bool(correct))), "ps_project")
        return out

    def grad_coeffs(self, lam, p):
        import torch
        self._check_field(lam, "lam")
        self._check_field(p, "p")
        g = torch.empty(self.nz, dtype=torch.float64, device=self.device)
        self._sync_stream()
        check(load().ps_grad_coeffs(self._h, _vp(lam.data_ptr()), _vp(p.data_ptr()),
                                    _vp(g.data_ptr())), "ps_grad_coeffs")
        return g

    def set_coeffs(self, rho):
        self.rho = np.ascontiguousarray(rho, dtype=np.float64)
        self._sync_stream()
        check(load().ps_plan_set_coeffs(self._h, _dptr(self.rho)), "ps_plan_set_coeffs")

    def info(self) -> dict:
        inf = PlanInfo()
        check(load().ps_plan_query(self._h, ctypes.byref(inf)), "ps_plan_query")
        return {f: getattr(inf, f) for f, _ in PlanInfo._fields_}

    def workspace_bytes(self) -> int:
        return int(load().ps_workspace_bytes(self._h))

    def autotune(self, reps: int = 5):
        """Time the kernel variants for this plan and keep the fastest (or
        apply an earlier choice for an equal plan from the tune cache)."""
        self._sync_stream()
        check(load().ps_plan_autotune(self._h, int(reps)), "ps_plan_autotune")


    def profile(self, enable: bool):
        """Start (clearing totals) or stop per-kernel event timing."""
        self._sync_stream()
        check(load().ps_plan_profile(self._h, int(bool(enable))), "ps_plan_profile")

    def profile_report(self) -> dict:
        """{kernel name: (total ms, launches)} for kernels launched while
        profiling was on (synchronises)."""
        out = {}
        i = 0
        lib = load()
        while True:
            name = ctypes.c_char_p()
            ms = ctypes.c_double()
            n = ctypes.c_int()
            if lib.ps_plan_profile_report(self._h, i, ctypes.byref(name), ctypes.byref(ms),
                                          ctypes.byref(n)) != 0:
                break
            if n.value:
                out[name.value.decode()] = (ms.value, n.value)
            i += 1
        return out

    def spectrum_shape(self):
        return (self.nz, self.nx // 2, self.ny)

    def forward_transform(self, rhs):
        import torch
        self._check_field(rhs, "rhs")
        cdt = torch.complex128 if self.dtype == torch.float64 else torch.complex64
        spec = torch.empty(self.spectrum_shape(), dtype=cdt, device=self.device)
        self._sync_stream()
        check(load().ps_forward_transform(self._h, _vp(rhs.data_ptr()), _vp(spec.data_ptr())),
              "ps_forward_transform")
        return spec

    def spectral_solve(self, spec, adjoint=False):
        self._sync_stream()
        check(load().ps_spectral_solve(self._h, _vp(spec.data_ptr()), int(bool(adjoint))),
              "ps_spectral_solve")
        return spec

    def inverse_transform(self, spec, out=None):
        out = self._out(out)
        self._sync_stream()
        check(load().ps_inverse_transform(self._h, _vp(spec.data_ptr()), _vp(out.data_ptr())),
              "ps_inverse_transform")
        return out

    def close(self):
        h, self._h = getattr(self, "_h", None), None
        if h is not None and h.value and _lib is not None:
            _lib.ps_plan_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _solve_fn():
    import torch

    class PoissonSolve(torch.autograd.Function):
        """p = S(b; rho) with gradients with respect to b and the per-level
        densities rho (the adjoint solve and the density-gradient kernel).
        Nothing spectral is saved between forward and backward: the
        backward pass recomputes through the adjoint solve."""

        @staticmethod
        def forward(ctx, b, rho, plan):
            rho_h = rho.detach().to("cpu", torch.float64).numpy().copy()
            if not np.array_equal(rho_h, plan.rho):
                plan.set_coeffs(rho_h)
            p = plan.solve(b.detach().contiguous())
            ctx.plan = plan
            ctx.rho_h = rho_h
            ctx.save_for_backward(p)
            ctx.rho_dtype = rho.dtype
            ctx.rho_device = rho.device
            return p

        @staticmethod
        def backward(ctx, gp):
            (p,) = ctx.saved_tensors
            plan = ctx.plan
            # the plan may have been used with other densities since this
            # forward: the adjoint and the density gradient need this
            # forward's operator, so its densities are set for them and the
            # plan's current ones restored afterwards
            current = plan.rho.copy()
            swap = not np.array_equal(current, ctx.rho_h)
            if swap:
                plan.set_coeffs(ctx.rho_h)
            try:
                lam = plan.solve_adjoint(gp.contiguous().to(plan.dtype))
                grho = None
                if ctx.needs_input_grad[1]:
                    grho = plan.grad_coeffs(lam, p).to(device=ctx.rho_device,
                                                       dtype=ctx.rho_dtype)
            finally:
                if swap:
                    plan.set_coeffs(current)
            return lam, grho, None

    return PoissonSolve


_poisson = None


def poisson_solve(b, rho, plan: Plan):
    """Differentiable solve: gradients flow to b and to rho (a 1-D tensor of
    the nz per-level densities)."""
    global _poisson
    if _poisson is None:
        _poisson = _solve_fn()
    return _poisson.apply(b, rho, plan)


class CGSolver:
    """Matrix-free Krylov solver on the same operator as Plan (the C ABI's
    ps_cg), FP64: method "cg" (on -D A) or "bicgstab" (on A, right
    preconditioned), preconditioner "none" or "jacobi".  solve() starts from
    x (or zeros) and returns (x, iterations, relative residual)."""

    PRECOND = {"none": 0, "jacobi": 1}
    METHOD = {"cg": 0, "bicgstab": 1}

    def __init__(self, nx, ny, nz, dx, dy, dz, rho, precond="jacobi", method="cg"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the pressure-solve library needs a GPU (no CPU fallback)")
        lib = load()
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.device = torch.device("cuda", torch.cuda.current_device())
        dz = np.ascontiguousarray(dz, dtype=np.float64)
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        h = _vp()
        check(lib.ps_cg_create(ctypes.byref(h), self.nx, self.ny, self.nz, float(dx), float(dy),
                               _dptr(dz), _dptr(rho), self.PRECOND[precond], _stream_handle()),
              "ps_cg_create")
        self._h = h
        check(lib.ps_cg_set_method(h, self.METHOD[method]), "ps_cg_set_method")
        self.method = method

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def solve(self, rhs, x=None, rtol=1e-8, max_iter=10000):
        import torch
        for t, nm in ((rhs, "rhs"),) + (((x, "x"),) if x is not None else ()):
            if t.dtype != torch.float64 or tuple(t.shape) != self.shape or not t.is_contiguous() \
                    or t.device != self.device:
                raise ValueError("%s must be a contiguous float64 tensor of shape %s on %s"
                                 % (nm, self.shape, self.device))
        if x is None:
            x = torch.zeros_like(rhs)
        it = ctypes.c_int()
        rr = ctypes.c_double()
        lib = load()
        check(lib.ps_cg_set_stream(self._h, _stream_handle()), "ps_cg_set_stream")
        check(lib.ps_cg_solve(self._h, _vp(rhs.data_ptr()), _vp(x.data_ptr()), float(rtol),
                              int(max_iter), ctypes.byref(it), ctypes.byref(rr)), "ps_cg_solve")
        return x, it.value, rr.value

    def close(self):
        h, self._h = getattr(self, "_h", None), None
        if h is not None and h.value and _lib is not None:
            _lib.ps_cg_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune_cache_save(path: str):
    check(load().ps_tune_cache_save(os.fsencode(path)), "ps_tune_cache_save")


def tune_cache_load(path: str):
    check(load().ps_tune_cache_load(os.fsencode(path)), "ps_tune_cache_load")


class BatchPlan:
    """Many independent solves of uneven sizes replayed from captured
    hipGraphs (the C ABI's ps_batch, mode PS_BATCH_LANES): the problems are
    dealt to ``lanes`` streams, largest first, each lane's solves captured
    into one graph, and the lane graphs launched side by side.  Every
    problem gives exactly its standalone Plan's result (same kernels).

    grids: sequence of workloads.Grid-like objects (nx, ny, nz, dx, dy, dz,
    rho); precision one of PRECISIONS.  The earlier modes "phases",
    "persistent" and "plans" are refused by the library."""

    MODES = {"phases": 0, "persistent": 1, "plans": 2, "lanes": 3}

    def __init__(self, grids, precision="fp32", mode="lanes", lanes=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the pressure-solve library needs a GPU (no CPU fallback)")
        lib = load()
        self.grids = list(grids)
        n = len(self.grids)
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.device = torch.device("cuda", torch.cuda.current_device())
        ia = lambda vals: (ctypes.c_int * n)(*vals)
        da = lambda vals: (ctypes.c_double * n)(*vals)
        self._dz = [np.ascontiguousarray(g.dz, dtype=np.float64) for g in self.grids]
        self._rho = [np.ascontiguousarray(g.rho, dtype=np.float64) for g in self.grids]
        dzp = (_D * n)(*[_dptr(a) for a in self._dz])
        rhop = (_D * n)(*[_dptr(a) for a in self._rho])
        h = _vp()
        check(lib.ps_batch_create(ctypes.byref(h), n, ia([g.nx for g in self.grids]),
                                  ia([g.ny for g in self.grids]), ia([g.nz for g in self.grids]),
                                  da([g.dx for g in self.grids]), da([g.dy for g in self.grids]),
                                  dzp, rhop, PRECISIONS[precision], _stream_handle()),
              "ps_batch_create")
        self._h = h
        try:
            check(lib.ps_batch_set_mode(h, self.MODES[mode]), "ps_batch_set_mode")
            if lanes is not None:
                self.set_lanes(lanes)
        except Exception:
            self.close()
            raise

    def set_lanes(self, lanes: int):
        check(load().ps_batch_set_lanes(self._h, int(lanes)), "ps_batch_set_lanes")

    def set_fp64_order(self, in_order: bool):
        """True (default): each problem's FP64 columns in order on its lane;
        False: each plan's own placement (forked onto its second stream)."""
        check(load().ps_batch_set_fp64_order(self._h, int(bool(in_order))),
              "ps_batch_set_fp64_order")

    def _ptrs(self, rhs, out):
        n = len(self.grids)
        for i, (b, p, g) in enumerate(zip(rhs, out, self.grids)):
            for t, nm in ((b, "rhs"), (p, "out")):
                if t.dtype != self.dtype or tuple(t.shape) != (g.nz, g.ny, g.nx) \
                        or not t.is_contiguous() or t.device != self.device:
                    raise ValueError("%s[%d] must be a contiguous %s tensor of shape %s on %s"
                                     % (nm, i, self.dtype, (g.nz, g.ny, g.nx), self.device))
        return ((_vp * n)(*[_vp(t.data_ptr()) for t in rhs]),
                (_vp * n)(*[_vp(t.data_ptr()) for t in out]))

    def solve(self, rhs, out):
        """Solve every problem: rhs and out are lists of tensors."""
        rp, op = self._ptrs(rhs, out)
        check(load().ps_batch_set_stream(self._h, _stream_handle()), "ps_batch_set_stream")
        check(load().ps_batch_solve(self._h, rp, op), "ps_batch_solve")
        return out

    def autotune(self, rhs, out, reps=3):
        rp, op = self._ptrs(rhs, out)
        check(load().ps_batch_set_stream(self._h, _stream_handle()), "ps_batch_set_stream")
        check(load().ps_batch_autotune(self._h, rp, op, int(reps)), "ps_batch_autotune")

    def status(self):
        """Synchronise the batch's streams; raise if a solve failed."""
        check(load().ps_batch_status(self._h), "ps_batch_status")

    def info(self) -> dict:
        c, l, o = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(load().ps_batch_query(self._h, ctypes.byref(c), ctypes.byref(l), ctypes.byref(o)),
              "ps_batch_query")
        return {"count": c.value, "lanes": l.value, "fp64_in_order": bool(o.value)}

    def close(self):
        h, self._h = getattr(self, "_h", None), None
        if h is not None and h.value and _lib is not None:
            _lib.ps_batch_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
