"""Helpers for the GPU tests: run a workload through the C-ABI library, run it through the
oracle, and compare the two."""
from __future__ import annotations

import sys

import numpy as np

import oracle as O
import workloads as W

KIND_NAMES = {1: "row", 2: "corrected", 3: "checksum", 4: "uncorrectable", 5: "window",
              6: "rollback", 7: "persistent", 8: "col", 9: "mem", 10: "mem_corrected",
              11: "mem_unlocated"}


def say(*args):
    """Name the case on stdout before a GPU step (flushed, so a fault still shows it)."""
    print("[gpu]", *args, flush=True)
    sys.stdout.flush()


def run_gpu(u0, taps, nsweeps, *, C=None, c_scalar=0.0, mode="online", eps=1e-12, period=10,
            csum="f64", auto_correct=True, plan=None, bc="clamp", bc_value=0.0, graph=False,
            chunks=None, max_events=1 << 16, autotune=False, input_check=True,
            correction="checksum", tile_x=0, tuning_cache=None):
    """Returns (final grid as numpy, events, report, stencil-shape)."""
    import torch
    from paper_1909_00709_amd import abft
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ut = torch.from_numpy(np.ascontiguousarray(u0)).cuda()
        Ct = torch.from_numpy(np.ascontiguousarray(C)).cuda() if C is not None else None
        S = abft.Stencil(ut, taps, C=Ct, c_scalar=c_scalar, bc=bc, bc_value=bc_value, mode=mode,
                         period=period, threshold=eps, csum=csum, auto_correct=auto_correct,
                         max_events=max_events, stream=stream, input_check=input_check,
                         correction=correction, tile_x=tile_x, tuning_cache=tuning_cache)
        try:
            if autotune:
                S.autotune()
            if plan is not None and len(plan):
                S.inject(plan)
            for n in (chunks or [nsweeps]):
                (S.step_graph if graph else S.step)(n)
            rep, ev = S.check()
            cur, t = S.current()
            out = cur.cpu().numpy()
            shape = S.launch_shape()
        finally:
            S.close()
    stream.synchronize()
    return out, ev, rep, shape


def run_oracle(u0, taps, nsweeps, *, C=None, c_scalar=0.0, mode="online", eps=1e-12, period=10,
               auto_correct=True, plan=None, bc="clamp", bc_value=0.0, dtype=None,
               input_check=True, recompute=False, tile_x=0):
    bcs = {"clamp": O.BC_CLAMP, "periodic": O.BC_PERIODIC, "constant": O.BC_CONSTANT}
    modes = {"none": O.MODE_NONE, "online": O.MODE_ONLINE, "offline": O.MODE_OFFLINE}
    dt = dtype if dtype is not None else (O.F32 if u0.dtype == np.float32 else O.F64)
    p = O.Problem(u0.shape, dt, taps, bc=bcs[bc], bc_value=bc_value, c_scalar=c_scalar)
    return p.run(u0, nsweeps, C, mode=modes[mode], period=period, eps=eps,
                 auto_correct=auto_correct, faults=plan, input_check=input_check,
                 recompute=recompute, tile_x=tile_x)


def event_keys(ev, kinds=(1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11), skip=None):
    """Set of (kind, sweep, z, y, x) for the selected kinds; skip(e) drops marginal entries."""
    out = set()
    for e in ev:
        k = int(e["kind"])
        if k not in kinds:
            continue
        if skip is not None and skip(e):
            continue
        out.add((KIND_NAMES[k], int(e["sweep"]), int(e["z"]), int(e["y"]), int(e["x"])))
    return out


def rel_errors(g, o):
    g = g.astype(np.float64)
    o = o.astype(np.float64)
    l2 = np.linalg.norm((g - o).ravel()) / max(np.linalg.norm(o.ravel()), 1e-300)
    mx = np.abs(g - o).max() / max(np.abs(o).max(), 1e-300)
    return l2, mx


def assert_grid_close(g, o, tol, what=""):
    assert np.all(np.isfinite(g)) == np.all(np.isfinite(o)), what
    l2, mx = rel_errors(g, o)
    assert l2 <= tol and mx <= tol, f"{what}: l2 {l2:.3e} max {mx:.3e} tol {tol:.1e}"


def corrected_values(ev):
    return {(int(e["sweep"]), int(e["z"]), int(e["y"]), int(e["x"])): float(e["b"])
            for e in ev if int(e["kind"]) == 2}


def guard_band_plan(plan, lo_bit, hi_bit):
    """Drop flips whose bit lies in [lo_bit, hi_bit]: their relative signal falls within
    [eps/4, 4*eps] of the threshold, where the GPU and the oracle may legitimately decide
    differently under rounding."""
    keep = [(p["bit"] < lo_bit) or (p["bit"] > hi_bit) for p in plan]
    return plan[np.array(keep, dtype=bool)] if len(plan) else plan
