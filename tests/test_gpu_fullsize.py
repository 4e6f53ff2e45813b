"""The 1024 x 1024 x 128 fp32 workload at full size, in the launch shapes the benchmark uses
(autotuned): parity with the oracle, and the offline run with 50 seeded flips."""
import json
import os
import tempfile

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import assert_grid_close, event_keys, rel_errors, run_gpu, run_oracle, say

pytestmark = pytest.mark.gpu
# where the run writes its result summary (JSON): $ABFT_TEST_OUT, else the system temp folder
OUT = os.environ.get("ABFT_TEST_OUT") or os.path.join(tempfile.gettempdir(), "abft_test_out")


def test_c5_online_parity_20_sweeps():
    u0, C = W.C5.inputs()
    plan = W.make_plan([(3, 64, 512, 1023, 30), (11, 0, 0, 0, 27), (17, 127, 1023, 511, 24)])
    say("C5 online parity")
    g, gev, grep, shape = run_gpu(u0, W.THERMAL_TAPS, 20, C=C, eps=1e-7, plan=plan,
                                  autotune=True)
    o, oev, ocnt = run_oracle(u0, W.THERMAL_TAPS, 20, C=C, eps=1e-7, plan=plan)
    assert event_keys(gev) == event_keys(oev)
    assert grep["corrected"] == 3
    assert_grid_close(g, o, 1e-5, "C5 online 20")


def test_c5_offline_parity_and_rollback():
    """20 sweeps (two windows) with a flip in each window: events equal to the oracle's and the
    result equal to the fault-free GPU run bitwise."""
    u0, C = W.C5.inputs()
    plan = W.make_plan([(4, 30, 700, 3, 29), (18, 99, 5, 1000, 26)])
    say("C5 offline parity")
    g, gev, grep, _ = run_gpu(u0, W.THERMAL_TAPS, 20, C=C, mode="offline", period=10,
                              eps=W.C5.eps, plan=plan)
    o, oev, ocnt = run_oracle(u0, W.THERMAL_TAPS, 20, C=C, mode="offline", period=10,
                              eps=W.C5.eps, plan=plan)
    assert event_keys(gev) == event_keys(oev)
    assert grep["rollbacks"] == 2
    clean = run_gpu(u0, W.THERMAL_TAPS, 20, C=C, mode="none")[0]
    assert np.array_equal(g, clean)
    assert_grid_close(g, o, 1e-5, "C5 offline 20")


def test_c5_offline_50_flips():
    """500 sweeps, offline every 10, 50 flips at distinct sweeps, bits 0..31.  Every window that
    holds a flip of bit >= 20 is rolled back; the result differs from the fault-free run only
    by the flips too small to see."""
    u0, C = W.C5.inputs()
    plan = W.c5_plan()
    say("C5 offline 50 flips")
    g, ev, rep, shape = run_gpu(u0, W.THERMAL_TAPS, W.C5.nsweeps, C=C, mode="offline",
                                period=W.C5.period, eps=W.C5.eps, plan=plan)
    clean = run_gpu(u0, W.THERMAL_TAPS, W.C5.nsweeps, C=C, mode="none")[0]
    # the fault-free offline run: no window flagged, noise well under the threshold
    ff, ffev, ffrep, _ = run_gpu(u0, W.THERMAL_TAPS, W.C5.nsweeps, C=C, mode="offline",
                                 period=W.C5.period, eps=W.C5.eps)
    assert ffrep["windows_flagged"] == 0 and ffrep["max_noise"] < 0.6 * W.C5.eps, ffrep
    assert np.array_equal(ff, clean)
    rolled = {int(e["sweep"]) for e in ev if e["kind"] == 6}
    per_bit = {}
    for p in plan:
        w0 = int(p["sweep"]) // W.C5.period * W.C5.period
        hit = w0 in rolled
        per_bit.setdefault(int(p["bit"]), []).append(bool(hit))
        if p["bit"] >= 20:
            assert hit, p
    assert rep["persistent"] == 0
    l2, mx = rel_errors(g, clean)
    nodet = [int(p["bit"]) for p in plan if int(p["sweep"]) // 10 * 10 not in rolled]
    summary = {"windows_flagged": rep["windows_flagged"], "rollbacks": rep["rollbacks"],
               "fault_free_max_noise": ffrep["max_noise"], "undetected_bits": sorted(nodet),
               "rel_l2_vs_fault_free": l2, "rel_max_vs_fault_free": mx,
               "detected_per_bit": {b: sum(v) for b, v in sorted(per_bit.items())},
               "planted_per_bit": {b: len(v) for b, v in sorted(per_bit.items())}}
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, "c5_offline_50_flips.json"), "w") as f:
        json.dump(summary, f, indent=1)
    print(json.dumps(summary))
    if not nodet:
        assert np.array_equal(g, clean)
    assert mx < 1e-3
