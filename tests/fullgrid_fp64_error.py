"""Error of the fp32 GPU grid of the 1024 x 1024 x 128 thermal workload (500 sweeps, offline
detection every 10 sweeps) against the fault-free fp64-storage oracle run, over the whole grid:
the paper's l2 norm of the difference (Section 5.1, Eq.(11)), the same relative to the
reference's norm, and the largest pointwise error relative to the reference's largest
magnitude.  Three GPU runs: fault-free; with the seeded flips that lie outside the guard band
(the oracle's record in tests/golden/c5_offline_50_flips.json); with all 50 seeded flips.

Not collected by pytest (the fp64 oracle run takes a minute or more of host time); run it on a
machine with the GPU:

    python tests/fullgrid_fp64_error.py OUT.json
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import workloads as W  # noqa: E402
from tests.gpu_util import error_vs, fp64_reference, run_gpu, say  # noqa: E402


def main(out_path):
    wl = W.C5
    u0, C = wl.inputs()
    plan = W.c5_plan()
    with open(os.path.join(HERE, "golden", "c5_offline_50_flips.json")) as f:
        meta = json.load(f)
    kept = plan[np.asarray(meta["skipped"]) == 0]
    t0 = time.time()
    ref = fp64_reference(u0, W.THERMAL_TAPS, wl.nsweeps, C=C, chunk=50,
                         name="fp64 reference, 1024x1024x128")
    res = {"workload": f"{wl.name}, {wl.nsweeps} sweeps, offline every {wl.period}, "
                       f"threshold {wl.eps}",
           "reference": "oracle, fp64 storage, fault-free", "oracle_seconds": time.time() - t0,
           "oracle_fp32_vs_fp64_whole_grid": meta["oracle_f32_vs_f64"]}
    for name, p in (("fault_free", None), ("flips_outside_guard_band", kept), ("all_50_flips", plan)):
        say("C5 offline", name)
        g, ev, rep, _ = run_gpu(u0, W.THERMAL_TAPS, wl.nsweeps, C=C, mode="offline",
                                period=wl.period, eps=wl.eps, plan=p)
        res[name] = dict(error_vs(g, ref), flips=0 if p is None else int(len(p)),
                         rollbacks=rep["rollbacks"], windows_flagged=rep["windows_flagged"],
                         max_noise=rep["max_noise"])
        print(json.dumps({name: res[name]}), flush=True)
    with open(out_path, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "fullgrid_fp64_error.json")
