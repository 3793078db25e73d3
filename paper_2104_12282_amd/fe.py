"""Thin ctypes binding of libfe_hip.so (include/fe_abi.h).

Argument marshalling only: torch tensors supply device memory and the stream;
every step of the computation runs in the HIP library.  Importing this module
does not need a GPU, but constructing a Problem does, and the library must be
built (``python -m paper_2104_12282_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("FE_HIP_LIB") or os.path.join(_PKG, "libfe_hip.so")

FE_OK, FE_EINVAL, FE_ENOMEM, FE_EDEVICE, FE_ENOTCONV, FE_EBREAKDOWN = 0, -1, -2, -3, -4, -5
PRECISION = {"fp64": 0, "fp32_ir": 1, "bf16_ir": 2, "bf16x3_ir": 3}
PRECOND = {"jacobi": 0, "gmg": 1}
PRECISION_NAME = {v: k for k, v in PRECISION.items()}
PRECOND_NAME = {v: k for k, v in PRECOND.items()}
STATUS_NAME = {0: "FE_OK", -1: "FE_EINVAL", -2: "FE_ENOMEM", -3: "FE_EDEVICE",
               -4: "FE_ENOTCONV", -5: "FE_EBREAKDOWN"}

# Every entry point declared in include/fe_abi.h.
ABI_SYMBOLS = ("fe_workspace_size", "fe_setup", "fe_apply_K", "fe_solve", "fe_solve_begin",
               "fe_solve_step", "fe_solve_end", "fe_sensitivity", "fe_sensitivity_adjoint", "fe_set_load",
               "fe_filter", "oc_update", "oc_update_noalloc", "fe_block_mean", "fe_extrapolate", "fe_set_mg_params", "fe_get_mg_params", "fe_set_mg_smoother", "fe_get_mg_smoother", "fe_set_float32_levels", "fe_set_coarse_fusion", "fe_set_profiling", "fe_set_cache_flush",
               "fe_kernel_stats", "fe_destroy", "fe_batch_workspace_size", "fe_batch_create", "fe_batch_setup_slot",
               "fe_batch_round_begin", "fe_batch_round_end", "fe_batch_round_ready", "fe_batch_destroy", "fe_onsg_num_params",
               "fe_onsg_workspace_size", "fe_onsg_create", "fe_onsg_add_samples", "fe_onsg_num_samples",
               "fe_onsg_train", "fe_onsg_predict", "fe_onsg_get_params", "fe_onsg_destroy", "fe_last_error")


class FEError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAME.get(status, status)}: {msg}")
        self.status = status


class fe_config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("h", C.c_double), ("E0", C.c_double), ("Emin", C.c_double),
                ("nu", C.c_double), ("penal", C.c_double), ("filter_r", C.c_double),
                ("precision", C.c_int32), ("precond", C.c_int32),
                ("mg_levels", C.c_int32), ("reserved", C.c_int32)]


class fe_solve_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("outer_iters", C.c_int32),
                ("rel_res", C.c_double), ("compliance", C.c_double)]


_lib = None


def load_library() -> C.CDLL:
    """Loads the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2104_12282_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P, D, I32, I64 = C.c_void_p, C.c_double, C.c_int32, C.c_int64
    lib.fe_workspace_size.argtypes = [C.POINTER(fe_config)]
    lib.fe_workspace_size.restype = C.c_size_t
    lib.fe_setup.argtypes = [C.POINTER(fe_config), P, P, P, C.c_size_t, P, C.POINTER(P)]
    lib.fe_apply_K.argtypes = [P, P, P, P, I32]
    lib.fe_solve.argtypes = [P, P, P, D, I32, C.POINTER(fe_solve_info)]
    lib.fe_solve_begin.argtypes = [P, P, P, D, I32]
    lib.fe_solve_step.argtypes = [P, C.POINTER(I32)]
    lib.fe_solve_end.argtypes = [P, C.POINTER(fe_solve_info)]
    lib.fe_sensitivity.argtypes = [P, P, P, P, P]
    lib.fe_sensitivity_adjoint.argtypes = [P, P, P, P, P]
    lib.fe_set_load.argtypes = [P, P]
    lib.fe_filter.argtypes = [P, P, P, I32]
    lib.oc_update.argtypes = [P, P, P, P, D, D, P, P]
    lib.oc_update_noalloc.argtypes = [I64, P, P, P, D, D, P, P, P]
    lib.fe_block_mean.argtypes = [P, P, I32, P]
    lib.fe_extrapolate.argtypes = [P, P, P, D]
    lib.fe_set_mg_params.argtypes = [P, I32, I32, D, D]
    lib.fe_set_float32_levels.argtypes = [P, I32]
    lib.fe_set_mg_smoother.argtypes = [P, I32, I32, D]
    lib.fe_get_mg_smoother.argtypes = [P, C.POINTER(I32), C.POINTER(I32), C.POINTER(D)]
    lib.fe_get_mg_params.argtypes = [P, C.POINTER(I32), C.POINTER(I32), C.POINTER(D), C.POINTER(D)]
    lib.fe_set_coarse_fusion.argtypes = [P, I32]
    lib.fe_set_profiling.argtypes = [P, I32]
    lib.fe_set_cache_flush.argtypes = [P, P, C.c_size_t]
    lib.fe_kernel_stats.argtypes = [P, I32, C.POINTER(I64), C.POINTER(D), C.POINTER(D)]
    lib.fe_destroy.argtypes = [P]
    lib.fe_destroy.restype = None
    lib.fe_batch_workspace_size.argtypes = [C.POINTER(fe_config), I32]
    lib.fe_batch_workspace_size.restype = C.c_size_t
    lib.fe_batch_create.argtypes = [C.POINTER(fe_config), I32, P, C.c_size_t, P, C.POINTER(P)]
    lib.fe_batch_setup_slot.argtypes = [P, I32, P, P, C.POINTER(P)]
    lib.fe_batch_round_begin.argtypes = [P]
    lib.fe_batch_round_end.argtypes = [P, C.POINTER(I32)]
    lib.fe_batch_round_ready.argtypes = [P, C.POINTER(I32)]
    lib.fe_batch_destroy.argtypes = [P]
    lib.fe_batch_destroy.restype = None
    lib.fe_onsg_num_params.argtypes = [I32, I32]
    lib.fe_onsg_num_params.restype = C.c_int64
    lib.fe_onsg_workspace_size.argtypes = [I32] * 7
    lib.fe_onsg_workspace_size.restype = C.c_size_t
    lib.fe_onsg_create.argtypes = [I32] * 7 + [P, P, C.c_size_t, P, C.POINTER(P)]
    lib.fe_onsg_add_samples.argtypes = [P, P, P, P]
    lib.fe_onsg_num_samples.argtypes = [P, C.POINTER(I64)]
    lib.fe_onsg_train.argtypes = [P, I32, P, D, I32, P]
    lib.fe_onsg_predict.argtypes = [P, P, P, P]
    lib.fe_onsg_get_params.argtypes = [P, P]
    lib.fe_onsg_destroy.argtypes = [P]
    lib.fe_onsg_destroy.restype = None
    lib.fe_last_error.argtypes = []
    lib.fe_last_error.restype = C.c_char_p
    for name in ("fe_setup", "fe_apply_K", "fe_solve", "fe_solve_begin", "fe_solve_step",
                 "fe_solve_end", "fe_sensitivity", "fe_filter",
                 "oc_update", "fe_set_mg_params", "fe_set_mg_smoother", "fe_get_mg_smoother", "fe_set_coarse_fusion", "fe_set_profiling", "fe_set_cache_flush", "fe_kernel_stats",
                 "fe_batch_create", "fe_batch_setup_slot", "fe_batch_round_begin", "fe_batch_round_end"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(status: int, allow=()):
    if status != FE_OK and status not in allow:
        raise FEError(status, load_library().fe_last_error().decode())
    return status


def _ptr(t: torch.Tensor | None, dtype=torch.float64):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor required")
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"contiguous {dtype} tensor required, got {t.dtype}")
    return C.c_void_p(t.data_ptr())


def make_config(nx, ny, nz, *, h=1.0, E0=1.0, Emin=1e-9, nu=0.3, penal=3.0, filter_r=1.5,
                precision="fp64", precond="jacobi", mg_levels=3) -> fe_config:
    return fe_config(nx, ny, nz, h, E0, Emin, nu, penal, filter_r, PRECISION[precision],
                     PRECOND[precond], mg_levels if precond == "gmg" else 0, 0)


def workspace_size(cfg: fe_config) -> int:
    return int(load_library().fe_workspace_size(C.byref(cfg)))


def oc_update_noalloc(x, dcx, dv, volfrac, move, x_new, change=None, stream=None):
    """The optimality-criteria update without a problem and without any
    allocation (include/fe_abi.h, oc_update_noalloc): x_new (and change, a
    one-element float64 tensor, if given) are written on `stream` (torch
    stream; the current stream of x's device by default) from the library's
    static scratch.  Asynchronous."""
    n = x.numel()
    if not (dcx.numel() == dv.numel() == x_new.numel() == n):
        raise ValueError("x, dcx, dv and x_new must have the same number of elements")
    if change is not None and change.numel() != 1:
        raise ValueError("change must hold one element")
    s = stream if stream is not None else torch.cuda.current_stream(x.device)
    _check(load_library().oc_update_noalloc(n, _ptr(x), _ptr(dcx), _ptr(dv), volfrac, move, _ptr(x_new),
                                            _ptr(change), C.c_void_p(s.cuda_stream)))
    return x_new


class Problem:
    """One FE problem (grid, material, load, supports) resident on the GPU."""

    def __init__(self, nx, ny, nz, f: torch.Tensor, fixed: torch.Tensor | None = None, *,
                 device="cuda:0", stream: torch.cuda.Stream | None = None, **cfg_kw):
        lib = load_library()
        self.nx, self.ny, self.nz = nx, ny, nz
        self.nelem = nx * ny * nz
        self.ndof = 3 * (nx + 1) * (ny + 1) * (nz + 1)
        self.cfg = make_config(nx, ny, nz, **cfg_kw)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = lib.fe_workspace_size(C.byref(self.cfg))
        if nbytes == 0:
            # validation failed: let fe_setup report why
            nbytes = 256
        self.ws_bytes = int(nbytes)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.f = f.to(self.device, torch.float64).contiguous()
        self.fixed = None if fixed is None else fixed.to(self.device, torch.uint8).contiguous()
        h = C.c_void_p()
        with torch.cuda.stream(self.stream):
            _check(lib.fe_setup(C.byref(self.cfg), _ptr(self.fixed, torch.uint8), _ptr(self.f),
                                C.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                                C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        self._owned = True

    @classmethod
    def _slot(cls, batch, handle, f, fixed):
        """A batch slot's problem: the handle belongs to the batch."""
        self = cls.__new__(cls)
        self.nx, self.ny, self.nz = batch.nx, batch.ny, batch.nz
        self.nelem = batch.nx * batch.ny * batch.nz
        self.ndof = 3 * (batch.nx + 1) * (batch.ny + 1) * (batch.nz + 1)
        self.cfg, self.device, self.stream = batch.cfg, batch.device, batch.stream
        self.ws, self.ws_bytes = batch.ws, batch.ws_bytes
        self.f, self.fixed = f, fixed
        self._h = handle
        self._owned = False
        return self

    # -- helpers -----------------------------------------------------------
    def _vec(self, n):
        return torch.empty(n, dtype=torch.float64, device=self.device)

    def close(self):
        if getattr(self, "_h", None):
            if getattr(self, "_owned", True):
                load_library().fe_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- ABI calls ---------------------------------------------------------
    def apply_K(self, rho, u, variant=0, out=None):
        y = self._vec(self.ndof) if out is None else out
        _check(load_library().fe_apply_K(self._h, _ptr(rho), _ptr(u), _ptr(y), variant))
        return y

    def solve(self, rho, u=None, rtol=1e-8, max_iters=100000, allow_notconv=False):
        if u is None:
            u = torch.zeros(self.ndof, dtype=torch.float64, device=self.device)
        info = fe_solve_info()
        allow = (FE_ENOTCONV,) if allow_notconv else ()
        st = _check(load_library().fe_solve(self._h, _ptr(rho), _ptr(u), rtol, max_iters,
                                            C.byref(info)), allow)
        return u, {"iters": info.iters, "outer_iters": info.outer_iters,
                   "rel_res": info.rel_res, "compliance": info.compliance, "status": st}

    # non-blocking form (continuous batching): begin, poll step() until True, end()
    def solve_begin(self, rho, u, rtol=1e-8, max_iters=100000):
        self._pending = (rho, u)  # keep the arrays alive while the solve runs
        _check(load_library().fe_solve_begin(self._h, _ptr(rho), _ptr(u), rtol, max_iters))

    def solve_step(self) -> bool:
        done = C.c_int32(0)
        _check(load_library().fe_solve_step(self._h, C.byref(done)))
        return bool(done.value)

    def solve_end(self, allow_notconv=False):
        info = fe_solve_info()
        allow = (FE_ENOTCONV,) if allow_notconv else ()
        st = _check(load_library().fe_solve_end(self._h, C.byref(info)), allow)
        self._pending = None
        return {"iters": info.iters, "outer_iters": info.outer_iters, "rel_res": info.rel_res,
                "compliance": info.compliance, "status": st}

    def sensitivity(self, rho, u, out=None, compliance_out=None):
        dc = self._vec(self.nelem) if out is None else out
        c = torch.zeros(1, dtype=torch.float64, device=self.device) if compliance_out is None \
            else compliance_out
        _check(load_library().fe_sensitivity(self._h, _ptr(rho), _ptr(u), _ptr(dc), _ptr(c)))
        return dc, c

    def sensitivity_adjoint(self, rho, u, lam, out=None):
        """-lam^T dr/drho of the adjoint gradient (include/fe_abi.h, fe_sensitivity_adjoint)."""
        g = self._vec(self.nelem) if out is None else out
        _check(load_library().fe_sensitivity_adjoint(self._h, _ptr(rho), _ptr(u), _ptr(lam), _ptr(g)))
        return g

    def set_load(self, f):
        """Replaces the load (fixed dofs ignored); blocks until its norm is known."""
        f = f.to(self.device, torch.float64).contiguous()
        _check(load_library().fe_set_load(self._h, _ptr(f)))
        self.f = f

    def linear_objective_gradient(self, rho, l, u=None, rtol=1e-8):
        """Gradient of J = l^T u(rho) by the adjoint method (Eq. 3): u solves
        K u = f (skipped when u is given), lam solves K lam = l (the load is
        swapped to l for that solve and restored), g = -lam^T dr/drho.
        Returns (g, u, lam)."""
        if u is None:
            u, _ = self.solve(rho, rtol=rtol)
        f = self.f
        self.set_load(l)
        try:
            lam, _ = self.solve(rho, rtol=rtol)
        finally:
            self.set_load(f)
        return self.sensitivity_adjoint(rho, u, lam), u, lam

    def filter(self, x, transpose=False, out=None):
        y = self._vec(self.nelem) if out is None else out
        _check(load_library().fe_filter(self._h, _ptr(x), _ptr(y), 1 if transpose else 0))
        return y

    def oc_update(self, x, dcx, dv, volfrac, move, out=None, change_out=None):
        xn = self._vec(self.nelem) if out is None else out
        ch = torch.zeros(1, dtype=torch.float64, device=self.device) if change_out is None \
            else change_out
        _check(load_library().oc_update(self._h, _ptr(x), _ptr(dcx), _ptr(dv), volfrac, move,
                                        _ptr(xn), _ptr(ch)))
        return xn, ch

    def extrapolate(self, u, u_hist, theta=1.0):
        """Initial guess of the next solve from the last two solutions:
        u <- u + theta (u - u_hist), u_hist <- the old u (include/fe_abi.h,
        fe_extrapolate)."""
        _check(load_library().fe_extrapolate(self._h, _ptr(u), _ptr(u_hist), float(theta)))

    def block_mean(self, z, nb, out=None):
        """Coarse-grained design variables of the two-scale scheme: the mean
        of z over each nb x nb x nb block of elements (include/fe_abi.h,
        fe_block_mean)."""
        n = (self.nx // nb) * (self.ny // nb) * (self.nz // nb) if nb >= 1 else 0
        zc = self._vec(max(1, n)) if out is None else out  # the library rejects a bad nb
        _check(load_library().fe_block_mean(self._h, _ptr(z), nb, _ptr(zc)))
        return zc

    def coarse_problem(self, nb, f_c, fixed_c=None, **cfg_kw):
        """The coarse problem of the two-scale scheme for block size nb: the
        (nx/nb, ny/nb, nz/nb) grid with element edge nb h and the same
        physical filter radius (filter_r / nb elements), the material of this
        problem, load f_c.  Keyword arguments override the solver settings
        (precision, precond, mg_levels)."""
        if nb < 1 or self.nx % nb or self.ny % nb or self.nz % nb:
            raise FEError(FE_EINVAL, "nb must be >= 1 and divide nx, ny and nz")
        c = self.cfg
        cx, cy, cz = self.nx // nb, self.ny // nb, self.nz // nb
        kw = dict(h=c.h * nb, E0=c.E0, Emin=c.Emin, nu=c.nu, penal=c.penal, filter_r=c.filter_r / nb,
                  precision=PRECISION_NAME[c.precision], precond=PRECOND_NAME[c.precond],
                  mg_levels=max(2, c.mg_levels))
        kw.update(cfg_kw)
        return Problem(cx, cy, cz, f_c, fixed_c, device=self.device, stream=self.stream, **kw)

    def set_mg_params(self, nu=1, coarse_sweeps=48, omega=0.35, coarse_ratio=5000.0):
        _check(load_library().fe_set_mg_params(self._h, nu, coarse_sweeps, omega, coarse_ratio))

    def mg_params(self):
        """The multigrid parameters in effect: nu, coarse_sweeps, omega, coarse_ratio."""
        nu, deg, om, ra = C.c_int32(), C.c_int32(), C.c_double(), C.c_double()
        _check(load_library().fe_get_mg_params(self._h, C.byref(nu), C.byref(deg), C.byref(om), C.byref(ra)))
        return {"nu": nu.value, "coarse_sweeps": deg.value, "omega": om.value, "coarse_ratio": ra.value}

    def set_mg_smoother(self, cheb_from_level=0, degree=4, ratio=30.0):
        """Chebyshev smoothing (degree steps on [lambda_max / ratio,
        1.02 lambda_max]) on levels cheb_from_level .. levels - 2 instead of
        damped Jacobi; 0: damped Jacobi on every level."""
        _check(load_library().fe_set_mg_smoother(self._h, cheb_from_level, degree, ratio))

    def mg_smoother(self):
        """The smoothing in effect: cheb_from_level (0: damped Jacobi), degree, ratio."""
        k, deg, ra = C.c_int32(), C.c_int32(), C.c_double()
        _check(load_library().fe_get_mg_smoother(self._h, C.byref(k), C.byref(deg), C.byref(ra)))
        return {"cheb_from_level": k.value, "degree": deg.value, "ratio": ra.value}

    def set_float32_levels(self, first_level):
        """Multigrid levels >= first_level of float64 solves in float32
        (0: the whole preconditioner, the default; the number of levels:
        none)."""
        _check(load_library().fe_set_float32_levels(self._h, first_level))

    def set_coarse_fusion(self, steps_per_launch=0):
        """Launch form of the Chebyshev steps (coarsest-level solve and
        middle-level smoothing; 0: chosen per level, the default; 5: three
        steps per launch on 3D tiles of 4 x 4 x 4 nodes; 3 / 4: pairs on 3D
        tiles of 4 x 4 x 4 / 4 x 4 x 8 nodes; 2: pairs on z-marching tiles;
        1: one step each)."""
        _check(load_library().fe_set_coarse_fusion(self._h, steps_per_launch))

    def set_profiling(self, on, mode=None):
        """Times finest-grid K*u launches: all forms, or only form `mode`
        (mode 7: the coarsest-level Chebyshev launches, one event pair per solve)."""
        sel = 0 if not on else (1 if mode is None else 2 + int(mode))
        _check(load_library().fe_set_profiling(self._h, sel))

    def set_cache_flush(self, buf: torch.Tensor | None):
        """Cold-cache timing of profiled launches: `buf` (a device tensor of at
        least 512 MB, overwritten) is streamed through before each one."""
        if buf is None:
            _check(load_library().fe_set_cache_flush(self._h, None, 0))
            return
        if not buf.is_cuda or not buf.is_contiguous():
            raise ValueError("contiguous device tensor required")
        _check(load_library().fe_set_cache_flush(self._h, C.c_void_p(buf.data_ptr()),
                                                 buf.numel() * buf.element_size()))

    def kernel_stats(self, reset=False):
        n, ms, b = C.c_int64(), C.c_double(), C.c_double()
        _check(load_library().fe_kernel_stats(self._h, 1 if reset else 0, C.byref(n), C.byref(ms),
                                              C.byref(b)))
        return {"launches": n.value, "total_ms": ms.value, "bytes_per_launch": b.value}


class Batch:
    """nslots designs of one configuration whose CG iterations share launches
    (include/fe_abi.h, fe_batch_*): slots are set up for new designs, their
    solves started with Problem.solve_begin, and advanced by rounds."""

    def __init__(self, nx, ny, nz, nslots, *, device="cuda:0", stream: torch.cuda.Stream | None = None,
                 **cfg_kw):
        lib = load_library()
        self.nx, self.ny, self.nz, self.nslots = nx, ny, nz, nslots
        cfg_kw.setdefault("precond", "gmg")
        self.cfg = make_config(nx, ny, nz, **cfg_kw)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ws_bytes = int(lib.fe_batch_workspace_size(C.byref(self.cfg), nslots)) or 256
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        with torch.cuda.stream(self.stream):
            _check(lib.fe_batch_create(C.byref(self.cfg), nslots, C.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                                       C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._b = h
        self.slots = [None] * nslots

    @staticmethod
    def workspace_bytes(nx, ny, nz, nslots, **cfg_kw) -> int:
        cfg_kw.setdefault("precond", "gmg")
        cfg = make_config(nx, ny, nz, **cfg_kw)
        return int(load_library().fe_batch_workspace_size(C.byref(cfg), nslots))

    def setup_slot(self, slot, f: torch.Tensor | None, fixed: torch.Tensor | None = None) -> Problem:
        f = None if f is None else f.to(self.device, torch.float64).contiguous()
        fixed = None if fixed is None else fixed.to(self.device, torch.uint8).contiguous()
        h = C.c_void_p()
        with torch.cuda.stream(self.stream):
            _check(load_library().fe_batch_setup_slot(self._b, slot, _ptr(fixed, torch.uint8), _ptr(f),
                                                      C.byref(h)))
        if self.slots[slot] is not None:
            self.slots[slot]._h = None  # the batch released the old handle
        self.slots[slot] = Problem._slot(self, h, f, fixed)
        return self.slots[slot]

    def round_begin(self):
        _check(load_library().fe_batch_round_begin(self._b))

    def round_end(self) -> int:
        n = C.c_int32()
        st = load_library().fe_batch_round_end(self._b, C.byref(n))
        if st != FE_OK:
            raise FEError(st, load_library().fe_last_error().decode())
        return n.value

    def round_ready(self) -> bool:
        """Whether the open round has completed on the device (no wait)."""
        n = C.c_int32()
        _check(load_library().fe_batch_round_ready(self._b, C.byref(n)))
        return bool(n.value)

    def close(self):
        if getattr(self, "_b", None):
            for s in self.slots:
                if s is not None:
                    s._h = None
            load_library().fe_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SyntheticGradientModel:
    """The network of the online synthetic gradients (include/fe_abi.h,
    fe_onsg_*): samples of the blocks of nb^3 elements of an (nx, ny, nz)
    grid, `width`-wide hidden layers, at most max_samples stored samples,
    mini-batches of `batch` rows."""

    def __init__(self, nx, ny, nz, nb, width, max_samples, batch, params, *, device="cuda:0",
                 stream: torch.cuda.Stream | None = None):
        lib = load_library()
        self.nx, self.ny, self.nz, self.nb, self.batch = nx, ny, nz, nb, batch
        self.n_params = int(lib.fe_onsg_num_params(nb, width))
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = int(lib.fe_onsg_workspace_size(nx, ny, nz, nb, width, max_samples, batch)) or 256
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        p = torch.as_tensor(params, dtype=torch.float64).to(self.device).contiguous()
        h = C.c_void_p()
        _check(lib.fe_onsg_create(nx, ny, nz, nb, width, max_samples, batch, _ptr(p),
                                  _ptr(self.ws, torch.uint8), nbytes, C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        torch.cuda.synchronize(self.device)  # the initial parameters are read
        self._h = h

    def add_samples(self, z, uc, g):
        _check(load_library().fe_onsg_add_samples(self._h, _ptr(z), _ptr(uc), _ptr(g)))

    @property
    def num_samples(self):
        n = C.c_int64()
        _check(load_library().fe_onsg_num_samples(self._h, C.byref(n)))
        return n.value

    def train(self, idx, lr0=5e-4, halve_every=500):
        """idx: int32 (steps, batch) sample indices; returns each step's loss."""
        idx = torch.as_tensor(idx, dtype=torch.int32).to(self.device).contiguous()
        if idx.dim() != 2 or idx.shape[1] != self.batch:
            raise ValueError(f"idx must be (steps, {self.batch})")
        losses = torch.empty(idx.shape[0], dtype=torch.float32, device=self.device)
        _check(load_library().fe_onsg_train(self._h, idx.shape[0], _ptr(idx, torch.int32), lr0, halve_every,
                                            _ptr(losses, torch.float32)))
        self._idx = idx  # alive until the stream has run the update
        return losses

    def predict(self, z, uc, out=None):
        g = torch.empty(self.nx * self.ny * self.nz, dtype=torch.float64, device=self.device) if out is None \
            else out
        _check(load_library().fe_onsg_predict(self._h, _ptr(z), _ptr(uc), _ptr(g)))
        return g

    def params(self):
        p = torch.empty(self.n_params, dtype=torch.float64, device=self.device)
        _check(load_library().fe_onsg_get_params(self._h, _ptr(p)))
        return p

    def close(self):
        if getattr(self, "_h", None):
            load_library().fe_onsg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
