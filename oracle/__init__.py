"""ctypes wrapper around the CPU oracle (abft_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package; the library under ``paper_1909_00709_amd`` never does.  The oracle
shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")
SOURCES = [os.path.join(HERE, "abft_oracle.c")]

F32, F64 = 0, 1
BC_CLAMP, BC_PERIODIC, BC_CONSTANT = 0, 1, 2
MODE_NONE, MODE_ONLINE, MODE_OFFLINE = 0, 1, 2
EV_ROW_FLAG, EV_CORRECTED, EV_CHECKSUM_FAULT, EV_UNCORRECTABLE = 1, 2, 3, 4
EV_WINDOW_FLAG, EV_ROLLBACK, EV_PERSISTENT, EV_COL_FLAG = 5, 6, 7, 8
EV_MEM_FLAG, EV_MEM_CORRECTED, EV_MEM_UNLOCATED = 9, 10, 11
FAULT_STORE, FAULT_MEMORY = 0, 1

EVENT_DTYPE = np.dtype([("sweep", "<i8"), ("kind", "<i4"), ("z", "<i4"), ("y", "<i4"),
                        ("x", "<i4"), ("a", "<f8"), ("b", "<f8")])
FAULT_INFO_DTYPE = np.dtype([("applied", "<i4"), ("skipped", "<i4"), ("before", "<f8"),
                             ("after", "<f8"), ("row_sum", "<f8"), ("col_sum", "<f8"),
                             ("signal", "<f8"), ("col_signal", "<f8")])
COUNTER_FIELDS = ("sweeps_done", "rows_flagged", "cols_flagged", "corrected",
                  "checksum_faults", "uncorrectable", "windows_checked", "windows_flagged",
                  "rollbacks", "persistent", "events_total", "mem_flagged", "mem_corrected",
                  "mem_unlocated")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11 + OpenMP, no contraction, no fast-math)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-o", tmp] + SOURCES + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Tap(ctypes.Structure):
    _fields_ = [("dx", ctypes.c_int32), ("dy", ctypes.c_int32), ("dz", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("w", ctypes.c_double)]


class _Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("ntaps", ctypes.c_int32), ("bc", ctypes.c_int32),
                ("taps", ctypes.POINTER(_Tap)), ("bc_value", ctypes.c_double),
                ("c_scalar", ctypes.c_double)]


class _Counters(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in COUNTER_FIELDS]


class _Guard(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double), ("hi", ctypes.c_double), ("info", ctypes.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, P = ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(_Problem)
        L.orc_validate.argtypes = [P]
        L.orc_sweep.argtypes = [P, vp, vp, vp]
        L.orc_row_checksums.argtypes = [P, vp, dp]
        L.orc_col_checksums.argtypes = [P, vp, dp]
        L.orc_weighted_row_checksums.argtypes = [P, vp, dp]
        L.orc_const_row_checksums.argtypes = [P, vp, dp]
        L.orc_const_col_checksums.argtypes = [P, vp, dp]
        L.orc_strip_width.argtypes = [P, ctypes.c_int]
        L.orc_row_strips.argtypes = [P, vp, dp]
        L.orc_col_strips.argtypes = [P, vp, dp]
        L.orc_predict_rows.argtypes = [P, dp, dp, dp, dp]
        L.orc_predict_cols.argtypes = [P, dp, dp, dp, dp]
        L.orc_detect.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_double, vp]
        L.orc_detect.restype = ctypes.c_int64
        L.orc_run.argtypes = [P, vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                              ctypes.c_int, ctypes.c_int, vp, vp, ctypes.c_int64, vp,
                              ctypes.c_int64, vp, ctypes.c_int64, ctypes.POINTER(_Counters),
                              ctypes.POINTER(_Guard)]
        L.orc_tile_checksums.argtypes = [P, vp, ctypes.c_int, dp]
        L.orc_const_tile_checksums.argtypes = [P, vp, ctypes.c_int, dp]
        L.orc_predict_tiles.argtypes = [P, dp, dp, vp, ctypes.c_int, dp]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_get_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Problem:
    """A stencil problem: grid shape (nz, ny, nx), storage dtype, taps, boundary rule."""

    def __init__(self, shape, dtype, taps, bc=BC_CLAMP, bc_value=0.0, c_scalar=0.0):
        nz, ny, nx = shape
        self.shape = (nz, ny, nx)
        self.dtype = dtype
        self.np_dtype = np.float32 if dtype == F32 else np.float64
        self.taps = list(taps)
        self._tap_arr = (_Tap * max(1, len(self.taps)))()
        for i, (dx, dy, dz, w) in enumerate(self.taps):
            self._tap_arr[i] = _Tap(dx, dy, dz, 0, float(w))
        self.c = _Problem(nx, ny, nz, dtype, len(self.taps), bc,
                          ctypes.cast(self._tap_arr, ctypes.POINTER(_Tap)), float(bc_value),
                          float(c_scalar))
        self.bc = bc
        self.bc_value = bc_value

    @property
    def ref(self):
        return ctypes.byref(self.c)

    def validate(self) -> int:
        return lib().orc_validate(self.ref)

    def _grid(self, a):
        a = np.ascontiguousarray(a, dtype=self.np_dtype)
        assert a.shape == self.shape, (a.shape, self.shape)
        return a

    def _const(self, C):
        return None if C is None else self._grid(C)

    # ---- single steps -------------------------------------------------------------------
    def sweep(self, u, C=None):
        u = self._grid(u)
        C = self._const(C)
        out = np.empty_like(u)
        lib().orc_sweep(self.ref, _ptr(C), _ptr(u), _ptr(out))
        return out

    def row_checksums(self, u):
        nz, ny, nx = self.shape
        B = np.empty((nz, ny))
        lib().orc_row_checksums(self.ref, _ptr(self._grid(u)), _ptr(B))
        return B

    def tile_checksums(self, u, T):
        nz, ny, nx = self.shape
        Bt = np.empty((nz, ny, nx // T))
        lib().orc_tile_checksums(self.ref, _ptr(self._grid(u)), T, _ptr(Bt))
        return Bt

    def const_tile_checksums(self, C, T):
        nz, ny, nx = self.shape
        cBt = np.empty((nz, ny, nx // T))
        lib().orc_const_tile_checksums(self.ref, _ptr(self._const(C)), T, _ptr(cBt))
        return cBt

    def predict_tiles(self, cBt, Bt, u, T):
        Bp = np.empty_like(np.asarray(Bt, dtype=np.float64))
        lib().orc_predict_tiles(self.ref, _ptr(np.ascontiguousarray(cBt, np.float64)),
                                _ptr(np.ascontiguousarray(Bt, np.float64)),
                                _ptr(self._grid(u)), T, _ptr(Bp))
        return Bp

    def weighted_row_checksums(self, u):
        nz, ny, nx = self.shape
        W = np.empty((nz, ny))
        lib().orc_weighted_row_checksums(self.ref, _ptr(self._grid(u)), _ptr(W))
        return W

    def col_checksums(self, u):
        nz, ny, nx = self.shape
        A = np.empty((nz, nx))
        lib().orc_col_checksums(self.ref, _ptr(self._grid(u)), _ptr(A))
        return A

    def const_row_checksums(self, C=None):
        nz, ny, nx = self.shape
        cB = np.empty((nz, ny))
        lib().orc_const_row_checksums(self.ref, _ptr(self._const(C)), _ptr(cB))
        return cB

    def const_col_checksums(self, C=None):
        nz, ny, nx = self.shape
        cA = np.empty((nz, nx))
        lib().orc_const_col_checksums(self.ref, _ptr(self._const(C)), _ptr(cA))
        return cA

    def row_strips(self, u):
        nz, ny, nx = self.shape
        r = lib().orc_strip_width(self.ref, 0)
        s = np.zeros((nz, ny, 2 * max(r, 1)))
        lib().orc_row_strips(self.ref, _ptr(self._grid(u)), _ptr(s))
        return s

    def col_strips(self, u):
        nz, ny, nx = self.shape
        r = lib().orc_strip_width(self.ref, 1)
        s = np.zeros((nz, nx, 2 * max(r, 1)))
        lib().orc_col_strips(self.ref, _ptr(self._grid(u)), _ptr(s))
        return s

    def predict_rows(self, cB, Bt, strips):
        Bp = np.empty_like(np.asarray(Bt, dtype=np.float64))
        lib().orc_predict_rows(self.ref, _ptr(np.ascontiguousarray(cB, np.float64)),
                               _ptr(np.ascontiguousarray(Bt, np.float64)),
                               _ptr(np.ascontiguousarray(strips, np.float64)), _ptr(Bp))
        return Bp

    def predict_cols(self, cA, At, strips):
        Ap = np.empty_like(np.asarray(At, dtype=np.float64))
        lib().orc_predict_cols(self.ref, _ptr(np.ascontiguousarray(cA, np.float64)),
                               _ptr(np.ascontiguousarray(At, np.float64)),
                               _ptr(np.ascontiguousarray(strips, np.float64)), _ptr(Ap))
        return Ap

    def predict_rows_from_grid(self, u, C=None):
        """Theorem 1 prediction of the next row checksums from grid u (its checksums + strips)."""
        return self.predict_rows(self.const_row_checksums(C), self.row_checksums(u),
                                 self.row_strips(u))

    def predict_cols_from_grid(self, u, C=None):
        return self.predict_cols(self.const_col_checksums(C), self.col_checksums(u),
                                 self.col_strips(u))

    # ---- whole runs -----------------------------------------------------------------------
    def run(self, u0, nsweeps, C=None, mode=MODE_ONLINE, period=10, eps=1e-12,
            auto_correct=True, faults=None, max_events=100000, input_check=True,
            recompute=False, tile_x=0, guard=None, info=None):
        """Returns (final grid, events structured array, counters dict).  Online mode:
        input_check also checks each sweep's input rows against the stored checksums;
        recompute corrects located points by evaluating them again from the sweep's input;
        tile_x > 0 keeps tile-local checksums of tile_x points (the input check is then off).
        guard = (lo, hi) leaves out the flips whose relative signal lies in [lo, hi] (see
        orc_guard); info, an array of FAULT_INFO_DTYPE with one entry per fault, receives
        what each flip did."""
        u_a = self._grid(u0).copy()
        u_b = np.empty_like(u_a)
        C = self._const(C)
        nf = 0 if faults is None else len(faults)
        fptr = None if nf == 0 else _ptr(np.ascontiguousarray(faults))
        ev = np.zeros(max_events, dtype=EVENT_DTYPE)
        cnt = _Counters()
        g = None
        if guard is not None or info is not None:
            if info is not None:
                assert info.dtype == FAULT_INFO_DTYPE and len(info) == nf and \
                    info.flags["C_CONTIGUOUS"]
            lo, hi = guard if guard is not None else (1.0, 0.0)
            g = _Guard(float(lo), float(hi), None if info is None or nf == 0
                       else info.ctypes.data_as(ctypes.c_void_p).value)
        rc = lib().orc_run(self.ref, _ptr(C), mode, period, eps, int(bool(auto_correct)),
                           (1 if input_check and not tile_x else 0) | (2 if recompute else 0),
                           int(tile_x), _ptr(u_a),
                           _ptr(u_b), nsweeps, fptr, nf,
                           _ptr(ev), max_events, ctypes.byref(cnt),
                           None if g is None else ctypes.byref(g))
        if rc != 0:
            raise ValueError(f"orc_run failed with code {rc}")
        counters = {f: getattr(cnt, f) for f in COUNTER_FIELDS}
        nev = min(counters["events_total"], max_events)
        return u_a, ev[:nev].copy(), counters


def detect(direct, pred, eps):
    direct = np.ascontiguousarray(direct, np.float64)
    pred = np.ascontiguousarray(pred, np.float64)
    flags = np.zeros(direct.shape, np.uint8)
    lib().orc_detect(direct.size, _ptr(direct), _ptr(pred), eps, _ptr(flags))
    return flags.astype(bool)


def set_threads(n: int):
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return lib().orc_get_threads()
