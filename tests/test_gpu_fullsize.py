"""The 1024 x 1024 x 128 fp32 workload at full size, in the launch shapes the benchmark uses
(autotuned): parity with the oracle, and the offline run with 50 seeded flips."""
import json
import os

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import (assert_grid_close, event_keys, rel_errors, run_gpu, run_oracle, say,
                            write_summary)

pytestmark = pytest.mark.gpu


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


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "c5_offline_50_flips")
# the stated sensitivity of this run: every window holding a flip of bit >= 17 rolls back
B_MIN_OFFLINE = 17


def _golden():
    """The oracle's run of this workload, stored by tests/golden/make_c5_offline.py."""
    with open(GOLDEN + ".json") as f:
        meta = json.load(f)
    return meta, np.load(GOLDEN + ".npz")


def test_c5_offline_50_flips_oracle_parity():
    """500 sweeps, offline every 10, the 50 seeded flips except those the oracle's run puts in
    the guard band [eps/4, 4 eps]: events and counters equal to the oracle's; the grid within
    1e-5 of the oracle's at 65 k seeded points and every flip site, every row sum within 1e-5;
    the error against the fault-free fp64-storage oracle run stated at the same points."""
    meta, gold = _golden()
    u0, C = W.C5.inputs()
    plan = W.c5_plan()
    assert meta["plan"] == [[int(p[k]) for k in ("sweep", "z", "y", "x", "bit")] for p in plan]
    kept = plan[np.asarray(meta["skipped"]) == 0]
    say("C5 offline oracle parity", len(kept), "of", len(plan))
    g, ev, rep, shape = run_gpu(u0, W.THERMAL_TAPS, W.C5.nsweeps, C=C, mode="offline",
                                period=W.C5.period, eps=W.C5.eps, plan=kept)
    gk = {(int(e["kind"]), int(e["sweep"]), int(e["z"]), int(e["y"]), int(e["x"])) for e in ev}
    ok = {tuple(e) for e in meta["events"]}
    assert gk == ok, (sorted(gk - ok), sorted(ok - gk))
    for k in ("windows_checked", "windows_flagged", "rollbacks", "persistent"):
        assert rep[k] == meta["counters"][k], k
    idx = gold["idx"]
    gs = g.ravel()[idx].astype(np.float64)
    o32 = gold["o32"].astype(np.float64)
    assert np.abs(gs - o32).max() <= 1e-5 * np.abs(o32).max()
    rows = g.astype(np.float64).sum(axis=2)
    orows = gold["rows32"].astype(np.float64)
    assert np.abs(rows - orows).max() <= 1e-5 * np.abs(orows).max()
    o64 = gold["o64"]
    d64 = gs - o64
    lay = rows.sum(axis=1)
    lay64 = np.asarray(meta["layer_sums_f64"])
    write_summary("c5_offline_oracle_parity.json", {
        "flips_run": int(len(kept)), "flips_left_out": int(len(plan) - len(kept)),
        "rollbacks": rep["rollbacks"], "windows_flagged": rep["windows_flagged"],
        "launch_shape": shape,
        "sampled_points": int(len(idx)),
        "vs_oracle_sampled_max_rel": float(np.abs(gs - o32).max() / np.abs(o32).max()),
        "vs_oracle_row_sums_max_rel": float(np.abs(rows - orows).max() / np.abs(orows).max()),
        "vs_fp64_oracle_sampled_max_rel": float(np.abs(d64).max() / np.abs(o64).max()),
        "vs_fp64_oracle_sampled_l2_rel": float(np.linalg.norm(d64) / np.linalg.norm(o64)),
        "vs_fp64_oracle_layer_sums_max_rel": float(np.abs(lay - lay64).max()
                                                   / np.abs(lay64).max()),
        "oracle_vs_fp64_oracle_whole_grid": meta["oracle_f32_vs_f64"]})


def test_c5_offline_50_flips():
    """500 sweeps, offline every 10, all 50 seeded flips at distinct sweeps, bits 0..31.
    Every window that holds a flip of bit >= 17 is rolled back; the result differs from the
    fault-free run only by the flips too small to see."""
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
        if p["bit"] >= B_MIN_OFFLINE:
            assert hit, p
    assert rep["persistent"] == 0
    l2, mx = rel_errors(g, clean)
    nodet = [int(p["bit"]) for p in plan if int(p["sweep"]) // 10 * 10 not in rolled]
    write_summary("c5_offline_50_flips.json", {
        "windows_flagged": rep["windows_flagged"], "rollbacks": rep["rollbacks"],
        "fault_free_max_noise": ffrep["max_noise"], "undetected_bits": sorted(nodet),
        "rel_l2_vs_fault_free": l2, "rel_max_vs_fault_free": mx,
        "detected_per_bit": {b: sum(v) for b, v in sorted(per_bit.items())},
        "planted_per_bit": {b: len(v) for b, v in sorted(per_bit.items())}})
    if not nodet:
        assert np.array_equal(g, clean)
    assert max(nodet, default=0) < B_MIN_OFFLINE
    assert mx < 1e-6
