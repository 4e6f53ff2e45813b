"""Helpers for the GPU tests: run a workload through the C-ABI library, run it through the
oracle, and compare the two."""
from __future__ import annotations

import json
import os
import sys
import tempfile
import time

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


# where the GPU tests write result summaries (JSON) and progress lines: $ABFT_TEST_OUT, else
# the system temp folder
OUT = os.environ.get("ABFT_TEST_OUT") or os.path.join(tempfile.gettempdir(), "abft_test_out")


def progress(name, msg):
    """One progress line of a long oracle run, appended to OUT/progress.log and printed."""
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, "progress.log"), "a") as f:
        f.write(f"{time.strftime('%H:%M:%S')} {name}: {msg}\n")
    print(f"[oracle] {name}: {msg}", flush=True)


def write_summary(name, summary):
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, name), "w") as f:
        json.dump(summary, f, indent=1)
    print(json.dumps(summary), flush=True)


def run_oracle(u0, taps, nsweeps, *, C=None, c_scalar=0.0, mode="online", eps=1e-12, period=10,
               auto_correct=True, plan=None, bc="clamp", bc_value=0.0, dtype=None,
               input_check=True, recompute=False, tile_x=0, guard=None, info=None,
               chunk=None, name=None):
    """The oracle's run of the same workload.  guard = (lo, hi) and info as in
    oracle.Problem.run.  chunk > 0 runs the sweeps in pieces of `chunk` (a multiple of the
    period offline), each starting from the last one's grid, with a progress line after each:
    the same run, since the checksums the next sweep predicts from, and offline the
    checkpoint, are those of the grid itself at a piece boundary."""
    bcs = {"clamp": O.BC_CLAMP, "periodic": O.BC_PERIODIC, "constant": O.BC_CONSTANT}
    modes = {"none": O.MODE_NONE, "online": O.MODE_ONLINE, "offline": O.MODE_OFFLINE}
    dt = dtype if dtype is not None else (O.F32 if u0.dtype == np.float32 else O.F64)
    p = O.Problem(u0.shape, dt, taps, bc=bcs[bc], bc_value=bc_value, c_scalar=c_scalar)
    kw = dict(mode=modes[mode], period=period, eps=eps, auto_correct=auto_correct,
              input_check=input_check, recompute=recompute, tile_x=tile_x, guard=guard)
    if not chunk or chunk >= nsweeps:
        return p.run(u0, nsweeps, C, faults=plan, info=info, **kw)
    assert mode != "offline" or chunk % period == 0, (chunk, period)
    assert auto_correct, "a halted offline run cannot be continued piecewise"
    plan = W.empty_plan(0) if plan is None else plan
    u = np.ascontiguousarray(u0)
    events, counters = [], None
    t0 = time.time()
    for s0 in range(0, nsweeps, chunk):
        n = min(chunk, nsweeps - s0)
        sel = np.nonzero((plan["sweep"] >= s0) & (plan["sweep"] < s0 + n))[0]
        part = plan[sel].copy()
        part["sweep"] -= s0
        pinfo = None if info is None else np.zeros(len(part), O.FAULT_INFO_DTYPE)
        u, ev, cnt = p.run(u, n, C, faults=part if len(part) else None, info=pinfo, **kw)
        if info is not None:
            info[sel] = pinfo
        ev = ev.copy()
        ev["sweep"] += s0
        events.append(ev)
        if counters is None:
            counters = dict(cnt)
        else:
            for k, v in cnt.items():
                counters[k] += v
        counters["sweeps_done"] = s0 + cnt["sweeps_done"]
        if name:
            progress(name, f"{s0 + n}/{nsweeps} sweeps, {time.time() - t0:.1f} s")
    return u, np.concatenate(events), counters


def guard_band(eps):
    """The band of relative signals in which two correct implementations may decide a flip
    differently under rounding: [eps/4, 4 eps]."""
    return (eps / 4.0, 4.0 * eps)


def guarded_oracle(u0, taps, nsweeps, plan, eps, **kw):
    """The oracle's run of `plan` with the flips inside the guard band left out.  Returns
    (grid, events, counters, kept plan, info): the kept plan is what the GPU runs to be
    compared event for event; info tells each flip's signal."""
    info = np.zeros(len(plan), O.FAULT_INFO_DTYPE)
    o, oev, ocnt = run_oracle(u0, taps, nsweeps, plan=plan, eps=eps, guard=guard_band(eps),
                              info=info, **kw)
    kept = plan[info["skipped"] == 0]
    return o, oev, ocnt, kept, info


def fp64_reference(u0, taps, nsweeps, *, C=None, chunk=None, name=None, **kw):
    """The fault-free oracle run of the same seeded inputs with fp64 storage (the grid and the
    constant term widened exactly, the weights rounded to fp64 instead of fp32)."""
    C64 = None if C is None else C.astype(np.float64)
    o, _, _ = run_oracle(u0.astype(np.float64), taps, nsweeps, C=C64, mode="none",
                         dtype=O.F64, chunk=chunk, name=name, **kw)
    return o


def error_vs(g, ref):
    """Error of grid g against a reference grid: the paper's l2 norm of the difference (Section
    5.1, Eq.(11)), the same relative to the reference's norm, and the largest pointwise error
    relative to the reference's largest magnitude."""
    g = g.astype(np.float64)
    ref = ref.astype(np.float64)
    d = (g - ref).ravel()
    l2 = float(np.sqrt(np.dot(d, d)))
    nref = float(np.linalg.norm(ref.ravel()))
    return {"l2_eq11": l2, "l2_rel": l2 / max(nref, 1e-300),
            "max_rel": float(np.abs(d).max() / max(np.abs(ref).max(), 1e-300))}


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
