"""MI355X (gfx950) Lagrange-flux solver: thin Python binding of the C ABI
in ``include/lagrangeflux.h`` (liblagrangeflux.so, built in-tree).

The binding only marshals arguments: every step of the solver runs in the
HIP kernels of the library.  PyTorch provides device memory and the
stream (``torch.cuda.current_stream()``).  There is no CPU fallback: if
the library is missing or no GPU is present, the calls raise.

State tensors: contiguous, shape (4 + n_species, ny, nx), dtype float64
(LF_F64) or float32 (LF_F32), on the solver's device, holding (rho, rho*u,
rho*v, rho*E) and then rho*y_k for the n_species passive mass fractions,
with x fastest.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblagrangeflux.so")

LF_OK, LF_ERR_ARG, LF_ERR_HIP, LF_ERR_NONPHYSICAL, LF_ERR_STATE, LF_ERR_TOO_LARGE = 0, 1, 2, 3, 4, 5
NOALLOC_SCRATCH_BYTES = 64 << 20  # LF_NOALLOC_SCRATCH_BYTES
LF_F64, LF_F32 = 0, 1
PERIODIC, TRANSMISSIVE = 0, 1
LF_MAX_SPECIES = 4
LF_RECON_PRIMITIVE, LF_RECON_CONSERVATIVE = 0, 1

# Names exported by the C ABI (include/lagrangeflux.h).
ABI_FUNCTIONS = ("lf_init", "lf_destroy", "lf_status_string", "lf_dt", "lf_step", "lf_step_save", "lf_step_halo",
                 "lf_stage", "lf_advance", "lf_residual", "lf_residual_vjp", "lf_adjoint_step",
                 "lf_adjoint_step_ustar", "lf_adjoint_step_noalloc", "lf_totals")
GHOST_ROWS = 4  # LF_GHOST_ROWS: rows a strip needs beyond each end for one step


class LFError(RuntimeError):
    def __init__(self, what: str, status: int):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} (status {status})")


class NonPhysicalState(LFError):
    """A state with rho <= 0, p <= 0 or a non-finite value was met.  From
    Solver.advance, ``t`` and ``steps`` tell how far the run got (the state
    produced by the last step is left in U)."""
    t = None
    steps = None


class lf_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double),
        ("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("beta", ctypes.c_double),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32), ("dtype", ctypes.c_int32),
        ("n_species", ctypes.c_int32), ("reconstruction", ctypes.c_int32),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load liblagrangeflux.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it first "
                              "(python -m paper_1607_08710_amd._build)")
        L = ctypes.CDLL(LIB_PATH)
        vp, d, i64 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int64
        L.lf_init.argtypes = [ctypes.POINTER(lf_params), ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_size_t)]
        L.lf_destroy.argtypes = [vp]
        L.lf_destroy.restype = None
        L.lf_status_string.argtypes = [ctypes.c_int]
        L.lf_status_string.restype = ctypes.c_char_p
        L.lf_dt.argtypes = [vp, vp, vp, vp, ctypes.POINTER(d)]
        L.lf_step.argtypes = [vp, vp, vp, d, vp, vp]
        L.lf_step_save.argtypes = [vp, vp, vp, vp, d, vp, vp]
        L.lf_step_halo.argtypes = [vp, vp, vp, vp, vp, d, vp, vp]
        L.lf_stage.argtypes = [vp, ctypes.c_int, vp, vp, vp, d, ctypes.c_int, vp, vp]
        L.lf_advance.argtypes = [vp, vp, d, d, i64, vp, vp, ctypes.POINTER(d), ctypes.POINTER(i64),
                                 ctypes.POINTER(d), i64]
        L.lf_residual.argtypes = [vp, vp, vp, vp, vp]
        L.lf_residual_vjp.argtypes = [vp, vp, vp, vp, vp, vp]
        L.lf_adjoint_step.argtypes = [vp, vp, d, vp, vp, vp, vp]
        L.lf_adjoint_step_ustar.argtypes = [vp, vp, vp, d, vp, vp, vp, vp]
        L.lf_adjoint_step_noalloc.argtypes = [vp, vp, d, vp, vp, vp]
        L.lf_totals.argtypes = [vp, vp, vp, vp, ctypes.POINTER(d)]
        for name in ("lf_init", "lf_dt", "lf_step", "lf_step_save", "lf_step_halo", "lf_stage", "lf_advance",
                     "lf_residual", "lf_residual_vjp", "lf_adjoint_step", "lf_adjoint_step_ustar",
                     "lf_adjoint_step_noalloc", "lf_totals"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().lf_status_string(int(status)).decode()


def _check(status: int, what: str):
    if status == LF_ERR_NONPHYSICAL:
        raise NonPhysicalState(what, status)
    if status != LF_OK:
        raise LFError(what, status)


@dataclass(frozen=True)
class Params:
    nx: int
    ny: int
    dx: float
    dy: float
    gamma: float = 1.4
    cfl: float = 0.5
    beta: float = 1.5
    bc_x: int = PERIODIC
    bc_y: int = PERIODIC
    dtype: int = LF_F64
    n_species: int = 0
    reconstruction: int = LF_RECON_PRIMITIVE

    def c(self) -> lf_params:
        return lf_params(self.nx, self.ny, self.dx, self.dy, self.gamma, self.cfl, self.beta,
                         self.bc_x, self.bc_y, self.dtype, self.n_species, self.reconstruction)


def init(params: Params):
    """lf_init: returns (ctx handle, workspace bytes).  No HIP call."""
    ctx = ctypes.c_void_p()
    ws = ctypes.c_size_t()
    p = params.c()
    _check(lib().lf_init(ctypes.byref(p), ctypes.byref(ctx), ctypes.byref(ws)), "lf_init")
    return ctx, ws.value


class Solver:
    """One context of the library plus its device workspace."""

    def __init__(self, params: Params, device="cuda"):
        import torch

        self.params = params
        dev = torch.device(device)
        if dev.type != "cuda":
            raise ValueError("the Lagrange-flux library runs on a HIP device only")
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.torch_dtype = torch.float64 if params.dtype == LF_F64 else torch.float32
        self.shape = (4 + params.n_species, params.ny, params.nx)
        self._ctx, self.ws_bytes = init(params)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx is not None and ctx.value and _lib is not None:
            _lib.lf_destroy(ctx)
            self._ctx = None

    # -- helpers -------------------------------------------------------------
    def _stream(self):
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _arg(self, t, name):
        if t.device != self.device or t.dtype != self.torch_dtype or tuple(t.shape) != self.shape \
                or not t.is_contiguous():
            raise ValueError(f"{name}: expected a contiguous {self.torch_dtype} tensor of shape "
                             f"{self.shape} on {self.device}, got {t.dtype} {tuple(t.shape)} on {t.device}")
        return ctypes.c_void_p(t.data_ptr())

    def empty_state(self):
        import torch
        return torch.empty(self.shape, dtype=self.torch_dtype, device=self.device)

    # -- C ABI ------------------------------------------------------------------
    def dt(self, U) -> float:
        out = ctypes.c_double()
        _check(lib().lf_dt(self._ctx, self._arg(U, "U"), ctypes.c_void_p(self.ws.data_ptr()),
                           self._stream(), ctypes.byref(out)), "lf_dt")
        return out.value

    def step(self, Un, Unp1, dt: float):
        _check(lib().lf_step(self._ctx, self._arg(Un, "Un"), self._arg(Unp1, "Unp1"), float(dt),
                             ctypes.c_void_p(self.ws.data_ptr()), self._stream()), "lf_step")

    def step_save(self, Un, Unp1, Ustar, dt: float):
        """One step into Unp1 that also writes the step's predictor state U*."""
        _check(lib().lf_step_save(self._ctx, self._arg(Un, "Un"), self._arg(Unp1, "Unp1"), self._arg(Ustar, "Ustar"),
                                  float(dt), ctypes.c_void_p(self.ws.data_ptr()), self._stream()), "lf_step_save")

    def step_halo(self, Un, ghost_lo, ghost_hi, Unp1, dt: float):
        """One step of this solver's grid as a strip of a larger one: the
        GHOST_ROWS rows below and above it are given, each a contiguous
        (fields, GHOST_ROWS, nx) tensor (ghost_lo row k is strip row
        k - GHOST_ROWS, ghost_hi row k is strip row ny + k)."""
        gshape = (self.shape[0], GHOST_ROWS, self.shape[2])
        for t, name in ((ghost_lo, "ghost_lo"), (ghost_hi, "ghost_hi")):
            if t.device != self.device or t.dtype != self.torch_dtype or tuple(t.shape) != gshape \
                    or not t.is_contiguous():
                raise ValueError(f"{name}: expected a contiguous {self.torch_dtype} tensor of shape {gshape} on "
                                 f"{self.device}, got {t.dtype} {tuple(t.shape)} on {t.device}")
        _check(lib().lf_step_halo(self._ctx, self._arg(Un, "Un"), ctypes.c_void_p(ghost_lo.data_ptr()),
                                  ctypes.c_void_p(ghost_hi.data_ptr()), self._arg(Unp1, "Unp1"), float(dt),
                                  ctypes.c_void_p(self.ws.data_ptr()), self._stream()), "lf_step_halo")

    def stage(self, stage: int, inp, out, dt: float, base=None, reduce: bool = False):
        """One Heun stage: 1 = predictor (out = in - dt R(in)), 2 = corrector
        (out = (base + in - dt R(in))/2)."""
        b = self._arg(base, "base") if base is not None else None
        _check(lib().lf_stage(self._ctx, int(stage), self._arg(inp, "in"), b, self._arg(out, "out"), float(dt),
                              1 if reduce else 0, ctypes.c_void_p(self.ws.data_ptr()), self._stream()),
               "lf_stage")

    def advance(self, U, t0: float, t_end: float, max_steps: int = 2**62, dts_capacity: int = 0):
        """Advance U in place; returns (t, steps, dts or None)."""
        t = ctypes.c_double()
        n = ctypes.c_int64()
        dts = np.empty(max(int(dts_capacity), 1), dtype=np.float64)
        dptr = dts.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if dts_capacity else None
        rc = lib().lf_advance(self._ctx, self._arg(U, "U"), float(t0), float(t_end), int(max_steps),
                              ctypes.c_void_p(self.ws.data_ptr()), self._stream(), ctypes.byref(t),
                              ctypes.byref(n), dptr, int(dts_capacity))
        if rc == LF_ERR_NONPHYSICAL:
            e = NonPhysicalState("lf_advance", rc)
            e.t, e.steps = t.value, n.value
            raise e
        _check(rc, "lf_advance")
        return t.value, n.value, (dts[: min(n.value, dts_capacity)].copy() if dts_capacity else None)

    def residual(self, U, R):
        _check(lib().lf_residual(self._ctx, self._arg(U, "U"), self._arg(R, "R"),
                                 ctypes.c_void_p(self.ws.data_ptr()), self._stream()), "lf_residual")

    def residual_vjp(self, U, g, out):
        _check(lib().lf_residual_vjp(self._ctx, self._arg(U, "U"), self._arg(g, "g"), self._arg(out, "out"),
                                     ctypes.c_void_p(self.ws.data_ptr()), self._stream()),
               "lf_residual_vjp")

    def adjoint_step(self, Un, dt: float, lam_np1, lam_n):
        _check(lib().lf_adjoint_step(self._ctx, self._arg(Un, "Un"), float(dt), self._arg(lam_np1, "lam_np1"),
                                     self._arg(lam_n, "lam_n"), ctypes.c_void_p(self.ws.data_ptr()),
                                     self._stream()), "lf_adjoint_step")

    def adjoint_step_ustar(self, Un, Ustar, dt: float, lam_np1, lam_n):
        """lf_adjoint_step with the step's U* given (from step_save)."""
        _check(lib().lf_adjoint_step_ustar(self._ctx, self._arg(Un, "Un"), self._arg(Ustar, "Ustar"), float(dt),
                                           self._arg(lam_np1, "lam_np1"), self._arg(lam_n, "lam_n"),
                                           ctypes.c_void_p(self.ws.data_ptr()), self._stream()),
               "lf_adjoint_step_ustar")

    def adjoint_step_noalloc(self, Un, dt: float, lam_np1, lam_n):
        """lf_adjoint_step without the workspace: U* and mu in the library's
        fixed device scratch (grids up to 1024^2 cells in FP64, 2 x 1024^2
        in FP32); allocates nothing.  Calls on one GPU must not overlap."""
        import torch
        with torch.cuda.device(self.device):  # the stream's device must be current
            _check(lib().lf_adjoint_step_noalloc(self._ctx, self._arg(Un, "Un"), float(dt),
                                                 self._arg(lam_np1, "lam_np1"), self._arg(lam_n, "lam_n"),
                                                 self._stream()), "lf_adjoint_step_noalloc")

    def totals(self, U) -> np.ndarray:
        out = (ctypes.c_double * self.shape[0])()
        _check(lib().lf_totals(self._ctx, self._arg(U, "U"), ctypes.c_void_p(self.ws.data_ptr()),
                               self._stream(), out), "lf_totals")
        return np.array(out[:])


from .rollout import LagrangeFluxRollout, checkpoint_spacing, rollout  # noqa: E402

__all__ = ["Params", "Solver", "LagrangeFluxRollout", "rollout", "checkpoint_spacing", "LFError", "NonPhysicalState",
           "PERIODIC", "TRANSMISSIVE", "LF_F64", "LF_F32", "lib", "init", "status_string"]
