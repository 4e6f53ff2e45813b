"""Python binding of libabft_stencil.so (include/abft_stencil.h).

Argument marshalling only: every step of the path runs in the library's HIP kernels.  The
functions named ``abft_*`` mirror the C entry points one to one; ``Stencil`` is a small
convenience wrapper that takes torch tensors (device memory and streams only).

The library is loaded from the package directory; there is no fallback.  If it is missing the
import of this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libabft_stencil.so")

# ---- constants (abft_stencil.h) --------------------------------------------------------------
ABFT_OK, ABFT_E_INVAL, ABFT_E_UNSUPPORTED, ABFT_E_NOMEM = 0, -1, -2, -3
ABFT_E_HIP, ABFT_E_STATE, ABFT_E_UNCORRECTABLE = -4, -5, -6
ABFT_F32, ABFT_F64 = 0, 1
ABFT_BC_CLAMP, ABFT_BC_PERIODIC, ABFT_BC_CONSTANT = 0, 1, 2
ABFT_MODE_NONE, ABFT_MODE_ONLINE, ABFT_MODE_OFFLINE = 0, 1, 2
ABFT_CSUM_F64, ABFT_CSUM_F32_COMP = 0, 1
ABFT_CORRECT_CHECKSUM, ABFT_CORRECT_RECOMPUTE = 0, 1
ABFT_EV_ROW_FLAG, ABFT_EV_CORRECTED, ABFT_EV_CHECKSUM_FAULT, ABFT_EV_UNCORRECTABLE = 1, 2, 3, 4
ABFT_EV_WINDOW_FLAG, ABFT_EV_ROLLBACK, ABFT_EV_PERSISTENT, ABFT_EV_COL_FLAG = 5, 6, 7, 8
ABFT_EV_MEM_FLAG, ABFT_EV_MEM_CORRECTED, ABFT_EV_MEM_UNLOCATED = 9, 10, 11
ABFT_FAULT_STORE, ABFT_FAULT_MEMORY = 0, 1

EXPORTED = (
    "abft_stencil_init", "abft_stencil_init_batch", "abft_stencil_step",
    "abft_stencil_step_graph", "abft_stencil_check", "abft_stencil_correct",
    "abft_stencil_current", "abft_stencil_checksums", "abft_stencil_inject",
    "abft_stencil_autotune", "abft_stencil_destroy", "abft_strerror", "abft_last_error",
    "abft_stencil_launch_shape", "abft_stencil_run_noalloc",
)
NOALLOC_SCRATCH_BYTES = 16 * 1024 * 1024  # ABFT_NOALLOC_SCRATCH_BYTES


class AbftTap(ctypes.Structure):
    _fields_ = [("dx", ctypes.c_int32), ("dy", ctypes.c_int32), ("dz", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("w", ctypes.c_double)]


class AbftProblem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("ntaps", ctypes.c_int32), ("bc", ctypes.c_int32),
                ("taps", ctypes.POINTER(AbftTap)), ("bc_value", ctypes.c_double),
                ("cterm", ctypes.c_void_p), ("cterm_scalar", ctypes.c_double),
                ("u0", ctypes.c_void_p), ("u1", ctypes.c_void_p), ("u2", ctypes.c_void_p)]


class AbftOptions(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("period", ctypes.c_int32),
                ("threshold", ctypes.c_double), ("csum", ctypes.c_int32),
                ("auto_correct", ctypes.c_int32), ("max_events", ctypes.c_int32),
                ("input_check", ctypes.c_int32), ("tuning_cache", ctypes.c_char_p),
                ("correction", ctypes.c_int32), ("tile_x", ctypes.c_int32)]


class AbftEvent(ctypes.Structure):
    _fields_ = [("sweep", ctypes.c_int64), ("kind", ctypes.c_int32), ("z", ctypes.c_int32),
                ("y", ctypes.c_int32), ("x", ctypes.c_int32), ("a", ctypes.c_double),
                ("b", ctypes.c_double), ("grid", ctypes.c_int32), ("pad", ctypes.c_int32)]


class AbftFault(ctypes.Structure):
    _fields_ = [("sweep", ctypes.c_int64), ("z", ctypes.c_int32), ("y", ctypes.c_int32),
                ("x", ctypes.c_int32), ("bit", ctypes.c_int32), ("attempt", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("kind", ctypes.c_int32), ("pad", ctypes.c_int32)]


REPORT_COUNTERS = ("sweeps_done", "rows_flagged", "cols_flagged", "corrected",
                   "checksum_faults", "uncorrectable", "windows_checked", "windows_flagged",
                   "rollbacks", "persistent", "events_total", "pending", "sweeps_skipped",
                   "mem_flagged", "mem_corrected", "mem_unlocated")


class AbftReport(ctypes.Structure):
    _fields_ = ([(f, ctypes.c_int64) for f in REPORT_COUNTERS] +
                [("max_noise", ctypes.c_double), ("nevents", ctypes.c_int32),
                 ("events_cap", ctypes.c_int32), ("events", ctypes.POINTER(AbftEvent))])


EVENT_DTYPE = np.dtype([("sweep", "<i8"), ("kind", "<i4"), ("z", "<i4"), ("y", "<i4"),
                        ("x", "<i4"), ("a", "<f8"), ("b", "<f8"), ("grid", "<i4"),
                        ("pad", "<i4")])
assert EVENT_DTYPE.itemsize == ctypes.sizeof(AbftEvent)
assert ctypes.sizeof(AbftFault) == 40

_ctx_p = ctypes.c_void_p


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with paper_1909_00709_amd/build.py "
            "(or __graft_entry__.build()); there is no fallback path")
    L = ctypes.CDLL(LIB_PATH)
    st = ctypes.c_int
    L.abft_stencil_init.argtypes = [ctypes.POINTER(AbftProblem), ctypes.POINTER(AbftOptions),
                                    ctypes.c_void_p, ctypes.POINTER(_ctx_p)]
    L.abft_stencil_init.restype = st
    L.abft_stencil_init_batch.argtypes = [ctypes.POINTER(AbftProblem), ctypes.c_int32,
                                          ctypes.POINTER(AbftOptions), ctypes.c_void_p,
                                          ctypes.POINTER(_ctx_p)]
    L.abft_stencil_init_batch.restype = st
    L.abft_stencil_step.argtypes = [_ctx_p, ctypes.c_int64]
    L.abft_stencil_step.restype = st
    L.abft_stencil_step_graph.argtypes = [_ctx_p, ctypes.c_int64]
    L.abft_stencil_step_graph.restype = st
    L.abft_stencil_check.argtypes = [_ctx_p, ctypes.POINTER(AbftReport)]
    L.abft_stencil_check.restype = st
    L.abft_stencil_correct.argtypes = [_ctx_p, ctypes.POINTER(AbftReport)]
    L.abft_stencil_correct.restype = st
    L.abft_stencil_current.argtypes = [_ctx_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(ctypes.c_int64)]
    L.abft_stencil_current.restype = st
    L.abft_stencil_checksums.argtypes = [_ctx_p, ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_void_p)]
    L.abft_stencil_checksums.restype = st
    L.abft_stencil_inject.argtypes = [_ctx_p, ctypes.c_void_p, ctypes.c_int32]
    L.abft_stencil_inject.restype = st
    L.abft_stencil_autotune.argtypes = [_ctx_p]
    L.abft_stencil_autotune.restype = st
    L.abft_stencil_destroy.argtypes = [_ctx_p]
    L.abft_stencil_destroy.restype = None
    L.abft_strerror.argtypes = [ctypes.c_int]
    L.abft_strerror.restype = ctypes.c_char_p
    L.abft_last_error.argtypes = [_ctx_p]
    L.abft_last_error.restype = ctypes.c_char_p
    L.abft_stencil_launch_shape.argtypes = [_ctx_p] + [ctypes.POINTER(ctypes.c_int32)] * 3
    L.abft_stencil_launch_shape.restype = st
    L.abft_stencil_run_noalloc.argtypes = [ctypes.POINTER(AbftProblem), ctypes.POINTER(AbftOptions),
                                           ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                           ctypes.c_void_p, ctypes.POINTER(AbftReport)]
    L.abft_stencil_run_noalloc.restype = st
    return L


LIB = _load()


# ---- one-to-one wrappers of the C entry points ----------------------------------------------
def abft_strerror(status: int) -> str:
    return LIB.abft_strerror(status).decode()


def abft_last_error(ctx) -> str:
    return LIB.abft_last_error(ctx).decode()


def abft_stencil_init(problem: AbftProblem, options: AbftOptions, stream: int):
    ctx = _ctx_p()
    s = LIB.abft_stencil_init(ctypes.byref(problem), ctypes.byref(options),
                              ctypes.c_void_p(stream), ctypes.byref(ctx))
    return s, ctx


def abft_stencil_init_batch(problems, options: AbftOptions, stream: int):
    arr = (AbftProblem * max(1, len(problems)))(*problems)
    ctx = _ctx_p()
    s = LIB.abft_stencil_init_batch(arr, len(problems), ctypes.byref(options),
                                    ctypes.c_void_p(stream), ctypes.byref(ctx))
    return s, ctx


def abft_stencil_step(ctx, nsweeps: int) -> int:
    return LIB.abft_stencil_step(ctx, nsweeps)


def abft_stencil_step_graph(ctx, nsweeps: int) -> int:
    return LIB.abft_stencil_step_graph(ctx, nsweeps)


def abft_stencil_check(ctx, report: AbftReport | None = None) -> int:
    return LIB.abft_stencil_check(ctx, ctypes.byref(report) if report is not None else None)


def abft_stencil_correct(ctx, report: AbftReport | None = None) -> int:
    return LIB.abft_stencil_correct(ctx, ctypes.byref(report) if report is not None else None)


def abft_stencil_current(ctx, grid: int = 0):
    p = ctypes.c_void_p()
    t = ctypes.c_int64()
    s = LIB.abft_stencil_current(ctx, grid, ctypes.byref(p), ctypes.byref(t))
    return s, p.value, t.value


def abft_stencil_checksums(ctx, grid: int = 0):
    p = ctypes.c_void_p()
    s = LIB.abft_stencil_checksums(ctx, grid, ctypes.byref(p))
    return s, p.value


def abft_stencil_inject(ctx, plan) -> int:
    """plan: numpy structured array with the abft_fault layout (40-byte records)."""
    if plan is None or len(plan) == 0:
        return LIB.abft_stencil_inject(ctx, None, 0)
    plan = np.ascontiguousarray(plan)
    assert plan.dtype.itemsize == ctypes.sizeof(AbftFault)
    return LIB.abft_stencil_inject(ctx, plan.ctypes.data_as(ctypes.c_void_p), len(plan))


def abft_stencil_autotune(ctx) -> int:
    return LIB.abft_stencil_autotune(ctx)


def abft_stencil_launch_shape(ctx):
    a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    s = LIB.abft_stencil_launch_shape(ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    return s, a.value, b.value, c.value


def abft_stencil_destroy(ctx) -> None:
    LIB.abft_stencil_destroy(ctx)


def abft_stencil_run_noalloc(problem: AbftProblem, options: AbftOptions, plan, nsweeps: int,
                             stream: int, report: AbftReport | None = None) -> int:
    """plan: numpy structured array with the abft_fault layout sorted by sweep, or None."""
    if plan is None or len(plan) == 0:
        fp, n = None, 0
    else:
        plan = np.ascontiguousarray(plan)
        assert plan.dtype.itemsize == ctypes.sizeof(AbftFault)
        fp, n = plan.ctypes.data_as(ctypes.c_void_p), len(plan)
    return LIB.abft_stencil_run_noalloc(ctypes.byref(problem), ctypes.byref(options), fp, n,
                                        nsweeps, ctypes.c_void_p(stream),
                                        ctypes.byref(report) if report is not None else None)


# ---- convenience wrapper over torch tensors ---------------------------------------------------
class AbftError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{abft_strerror(status)} ({status}): {msg}")
        self.status = status


_BC = {"clamp": ABFT_BC_CLAMP, "periodic": ABFT_BC_PERIODIC, "constant": ABFT_BC_CONSTANT}
_MODE = {"none": ABFT_MODE_NONE, "online": ABFT_MODE_ONLINE, "offline": ABFT_MODE_OFFLINE}
_CSUM = {"f64": ABFT_CSUM_F64, "f32comp": ABFT_CSUM_F32_COMP}
_CORRECTION = {"checksum": ABFT_CORRECT_CHECKSUM, "recompute": ABFT_CORRECT_RECOMPUTE}


def make_problem(shape, dtype_code, taps, u0_ptr, u1_ptr, u2_ptr=None, cterm_ptr=None,
                 cterm_scalar=0.0, bc="clamp", bc_value=0.0):
    nz, ny, nx = shape
    tap_arr = (AbftTap * len(taps))(*[AbftTap(int(dx), int(dy), int(dz), 0, float(w))
                                      for dx, dy, dz, w in taps])
    p = AbftProblem(nx, ny, nz, dtype_code, len(taps), _BC[bc] if isinstance(bc, str) else bc,
                    ctypes.cast(tap_arr, ctypes.POINTER(AbftTap)), float(bc_value),
                    cterm_ptr, float(cterm_scalar), u0_ptr, u1_ptr, u2_ptr)
    p._keep = tap_arr  # keep the tap array alive with the struct
    return p


def make_options(mode="online", period=10, threshold=1e-7, csum="f64", auto_correct=True,
                 max_events=4096, tuning_cache=None, input_check=False, correction="checksum",
                 tile_x=0):
    return AbftOptions(_MODE[mode] if isinstance(mode, str) else mode, int(period),
                       float(threshold), _CSUM[csum] if isinstance(csum, str) else csum,
                       int(bool(auto_correct)), int(max_events), int(bool(input_check)),
                       tuning_cache.encode() if tuning_cache else None,
                       _CORRECTION[correction] if isinstance(correction, str) else correction,
                       int(tile_x))


class Stencil:
    """One protected grid on the GPU.  u0 is a contiguous device tensor [nz][ny][nx] (float32
    or float64) holding u^0; the work buffers are allocated with torch.  input_check (online
    mode) also checks each sweep's input rows against their stored checksums and repairs
    faults that arose in memory between sweeps; it is on unless turned off."""

    def __init__(self, u0, taps, *, C=None, c_scalar=0.0, bc="clamp", bc_value=0.0,
                 mode="online", period=10, threshold=1e-7, csum="f64", auto_correct=True,
                 max_events=4096, stream=None, tuning_cache=None, input_check=True,
                 correction="checksum", tile_x=0):
        import torch
        if not u0.is_cuda or not u0.is_contiguous() or u0.dim() != 3:
            raise ValueError("u0 must be a contiguous 3D device tensor [nz][ny][nx]")
        if u0.dtype not in (torch.float32, torch.float64):
            raise ValueError("u0 must be float32 or float64")
        if C is not None and (C.shape != u0.shape or C.dtype != u0.dtype or not C.is_cuda
                              or not C.is_contiguous()):
            raise ValueError("C must match u0 (shape, dtype, device, contiguous)")
        self.torch = torch
        self.dtype_code = ABFT_F32 if u0.dtype == torch.float32 else ABFT_F64
        self.bufs = [u0, torch.empty_like(u0)]
        if mode == "offline":
            self.bufs.append(torch.empty_like(u0))
        self.C = C
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.max_events = max_events
        self.problem = make_problem(tuple(u0.shape), self.dtype_code, taps, u0.data_ptr(),
                                    self.bufs[1].data_ptr(),
                                    self.bufs[2].data_ptr() if len(self.bufs) > 2 else None,
                                    C.data_ptr() if C is not None else None, c_scalar, bc,
                                    bc_value)
        self.options = make_options(mode, period, threshold, csum, auto_correct, max_events,
                                    tuning_cache, input_check and not tile_x, correction, tile_x)
        s, ctx = abft_stencil_init(self.problem, self.options, self.stream.cuda_stream)
        if s != ABFT_OK:
            raise AbftError(s, abft_last_error(None))
        self.ctx = ctx

    def _chk(self, s):
        if s != ABFT_OK:
            raise AbftError(s, abft_last_error(self.ctx))
        return s

    def step(self, n: int):
        return self._chk(abft_stencil_step(self.ctx, n))

    def step_graph(self, n: int):
        return self._chk(abft_stencil_step_graph(self.ctx, n))

    def _report(self, fn):
        ev = (AbftEvent * max(1, self.max_events))()
        rep = AbftReport()
        rep.events = ctypes.cast(ev, ctypes.POINTER(AbftEvent))
        rep.events_cap = self.max_events
        s = fn(self.ctx, rep)
        out = {f: getattr(rep, f) for f in REPORT_COUNTERS}
        out["max_noise"] = rep.max_noise
        n = rep.nevents
        arr = np.frombuffer(ev, dtype=EVENT_DTYPE, count=len(ev))[:n].copy()
        return s, out, arr

    def check(self):
        s, rep, ev = self._report(abft_stencil_check)
        self._chk(s)
        return rep, ev

    def correct(self):
        """Returns (status, report, events); status may be ABFT_E_UNCORRECTABLE."""
        s, rep, ev = self._report(abft_stencil_correct)
        if s not in (ABFT_OK, ABFT_E_UNCORRECTABLE):
            self._chk(s)
        return s, rep, ev

    def current(self):
        s, ptr, t = abft_stencil_current(self.ctx, 0)
        self._chk(s)
        for b in self.bufs:
            if b.data_ptr() == ptr:
                return b, t
        raise RuntimeError("current grid is not one of the context's buffers")

    def checksum_plane_ptr(self):
        s, ptr = abft_stencil_checksums(self.ctx, 0)
        self._chk(s)
        return ptr

    def inject(self, plan):
        return self._chk(abft_stencil_inject(self.ctx, plan))

    def autotune(self):
        return self._chk(abft_stencil_autotune(self.ctx))

    def launch_shape(self):
        s, rows, planes, lanes = abft_stencil_launch_shape(self.ctx)
        self._chk(s)
        return rows, planes, lanes

    def close(self):
        if getattr(self, "ctx", None):
            abft_stencil_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent grids swept together (abft_stencil_init_batch).  grids is a list of
    (u0, C) pairs of contiguous device tensors (C may be None); all grids share the dtype, the
    taps and the options."""

    def __init__(self, grids, taps, *, c_scalar=0.0, bc="clamp", bc_value=0.0, mode="online",
                 threshold=1e-7, csum="f64", auto_correct=True, max_events=4096, stream=None,
                 correction="checksum", input_check=True):
        import torch
        self.torch = torch
        self.bufs, self.Cs, problems = [], [], []
        for u0, C in grids:
            if not u0.is_cuda or not u0.is_contiguous() or u0.dim() != 3:
                raise ValueError("each u0 must be a contiguous 3D device tensor")
            code = ABFT_F32 if u0.dtype == torch.float32 else ABFT_F64
            pair = [u0, torch.empty_like(u0)]
            self.bufs.append(pair)
            self.Cs.append(C)
            problems.append(make_problem(tuple(u0.shape), code, taps, u0.data_ptr(),
                                         pair[1].data_ptr(), None,
                                         C.data_ptr() if C is not None else None, c_scalar,
                                         bc, bc_value))
        self.problems = problems
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.max_events = max_events
        self.options = make_options(mode, 1, threshold, csum, auto_correct, max_events,
                                    correction=correction, input_check=input_check)
        s, ctx = abft_stencil_init_batch(problems, self.options, self.stream.cuda_stream)
        if s != ABFT_OK:
            raise AbftError(s, abft_last_error(None))
        self.ctx = ctx

    _chk = Stencil._chk
    step = Stencil.step
    step_graph = Stencil.step_graph
    _report = Stencil._report
    check = Stencil.check
    correct = Stencil.correct
    inject = Stencil.inject
    autotune = Stencil.autotune
    launch_shape = Stencil.launch_shape
    close = Stencil.close
    __del__ = Stencil.__del__

    def current(self, g: int):
        s, ptr, t = abft_stencil_current(self.ctx, g)
        self._chk(s)
        for b in self.bufs[g]:
            if b.data_ptr() == ptr:
                return b, t
        raise RuntimeError("current grid is not one of the grid's buffers")
