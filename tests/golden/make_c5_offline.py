"""Writes the oracle's results for the 1024 x 1024 x 128 fp32 thermal workload: 500 sweeps,
offline detection every 10 sweeps (Section 4), threshold 1e-6, the 50 seeded flips of
`workloads.c5_plan()` (Section 5.1 fault model), for the full-size GPU parity test.

Calls only `oracle/` (and `workloads/` for the seeded inputs).  The oracle runs once with the
guard band [eps/4, 4 eps] (flips whose relative signal lies there are left out and recorded as
such: under rounding two correct implementations may decide them either way), and once
fault-free with fp64 storage (the grid and constant term widened exactly, the weights rounded
to fp64), the reference the fp32 error is stated against.

Written: c5_offline_50_flips.json (the plan's guard records, the events, the counters, per-
layer sums and the oracle-vs-fp64-oracle error over the whole grid) and
c5_offline_50_flips.npz (a seeded sample of points of both final grids, with every flip site
and its row ends, and the fp32 run's row sums as fp32).

    python tests/golden/make_c5_offline.py      # about 25 minutes on 8 cores
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

NAME = "c5_offline_50_flips"
SAMPLE_SEED = 5005
NSAMPLES = 1 << 16


def sample_indices(shape, plan):
    """Flat indices of the sampled points: NSAMPLES drawn from rng(SAMPLE_SEED), plus each flip
    site and the two ends of its row, sorted and unique."""
    nz, ny, nx = shape
    rng = np.random.default_rng(SAMPLE_SEED)
    idx = list(rng.integers(0, nz * ny * nx, NSAMPLES))
    for p in plan:
        base = (int(p["z"]) * ny + int(p["y"])) * nx
        idx += [base + int(p["x"]), base, base + nx - 1]
    return np.unique(np.asarray(idx, np.int64))


def error_vs(g, ref):
    d = (g.astype(np.float64) - ref.astype(np.float64)).ravel()
    l2 = float(np.sqrt(np.dot(d, d)))
    nref = float(np.linalg.norm(ref.astype(np.float64).ravel()))
    return {"l2_eq11": l2, "l2_rel": l2 / nref,
            "max_rel": float(np.abs(d).max() / np.abs(ref).max())}


def main():
    wl = W.C5
    u0, C = wl.inputs()
    plan = W.c5_plan()
    eps = wl.eps
    t0 = time.time()
    p32 = O.Problem(wl.shape, O.F32, W.THERMAL_TAPS)
    info = np.zeros(len(plan), O.FAULT_INFO_DTYPE)
    o32, ev, cnt = p32.run(u0, wl.nsweeps, C, mode=O.MODE_OFFLINE, period=wl.period, eps=eps,
                           faults=plan, guard=(eps / 4, 4 * eps), info=info)
    print(f"guarded fp32 run: {time.time() - t0:.0f} s", flush=True)
    p64 = O.Problem(wl.shape, O.F64, W.THERMAL_TAPS)
    o64, ev64, cnt64 = p64.run(u0.astype(np.float64), wl.nsweeps, C.astype(np.float64),
                               mode=O.MODE_NONE)
    print(f"fp64 reference: {time.time() - t0:.0f} s", flush=True)
    idx = sample_indices(wl.shape, plan)
    rows32 = o32.astype(np.float64).sum(axis=2)
    meta = {
        "workload": wl.name, "nsweeps": wl.nsweeps, "period": wl.period, "eps": eps,
        "guard": [eps / 4, 4 * eps],
        "plan": [[int(p[k]) for k in ("sweep", "z", "y", "x", "bit")] for p in plan],
        "skipped": [int(v) for v in info["skipped"]],
        "signal": [float(v) for v in info["signal"]],
        "before": [float(v) for v in info["before"]],
        "after": [float(v) for v in info["after"]],
        "events": [[int(e["kind"]), int(e["sweep"]), int(e["z"]), int(e["y"]), int(e["x"])]
                   for e in ev],
        "counters": {k: int(v) for k, v in cnt.items()},
        "layer_sums_f32": [float(v) for v in rows32.sum(axis=1)],
        "layer_sums_f64": [float(v) for v in o64.sum(axis=(1, 2))],
        "oracle_f32_vs_f64": error_vs(o32, o64),
        "sample_seed": SAMPLE_SEED, "nsamples": int(len(idx)),
    }
    with open(os.path.join(HERE, NAME + ".json"), "w") as f:
        json.dump(meta, f, indent=0)
    np.savez_compressed(os.path.join(HERE, NAME + ".npz"), idx=idx,
                        o32=o32.ravel()[idx], o64=o64.ravel()[idx],
                        rows32=rows32.astype(np.float32))
    print(json.dumps({k: meta[k] for k in ("counters", "oracle_f32_vs_f64", "skipped")}))


if __name__ == "__main__":
    main()
