"""Fault campaign on the 512 x 512 x 64 fp32 thermal grid (one flip per sweep, bit = sweep mod 32,
1000 sweeps), both row-checksum accumulations, plus a fault-free 1000-sweep run for the false
positive rate (32.8 million row tests per accumulation mode).

Smallest detectable bit.  A flip of mantissa bit b of a value v with exponent e changes it by
2^(e-23+b); the row sum S of 512 values lies in [512*80, 512*331] over this run (the field
relaxes from 320..330 towards 80), and e is 6..8.  The relative signal is therefore at least
2^(b-17)/169472, which exceeds eps = 1e-7 for every b >= 12: bits 12..31 must all be detected,
located at their exact site and corrected.  It is at most 2^(b-15)/40960, below eps/4 for
b <= 5: bits 0..5 are never seen.  Bits 6..11 depend on the value at the time of the flip.
"""
import collections

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import (assert_grid_close, error_vs, event_keys, fp64_reference,
                            guarded_oracle, run_gpu, say, write_summary)

pytestmark = pytest.mark.gpu

B_MIN_GUARANTEED = 12
B_MAX_NEVER = 5


@pytest.fixture(scope="module")
def c3_oracle():
    """The oracle's runs of the whole campaign, made once for both accumulations: the 1000
    seeded flips with those in the guard band [eps/4, 4 eps] left out, and the fault-free
    run with fp64 storage (the reference the fp32 error is stated against)."""
    nz, ny, nx = W.C3.shape
    u0, C = W.thermal_grid(nx, ny, nz, np.float32)
    plan = W.c3_campaign()
    o, oev, ocnt, kept, info = guarded_oracle(u0, W.THERMAL_TAPS, W.C3.nsweeps, plan, W.C3.eps,
                                              C=C, chunk=100, name="C3 campaign")
    ref = fp64_reference(u0, W.THERMAL_TAPS, W.C3.nsweeps, C=C, chunk=250,
                         name="C3 fp64 reference")
    return {"u0": u0, "C": C, "plan": plan, "grid": o, "events": oev, "counters": ocnt,
            "kept": kept, "info": info, "ref64": ref}


def _summary(plan, ev):
    planted = {(int(p["sweep"]), int(p["z"]), int(p["y"]), int(p["x"])): int(p["bit"])
               for p in plan}
    rows = {(int(e["sweep"]), int(e["z"]), int(e["y"])) for e in ev if e["kind"] == 1}
    fixed = {(int(e["sweep"]), int(e["z"]), int(e["y"]), int(e["x"])) for e in ev
             if e["kind"] == 2}
    planted_rows = {k[:3] for k in planted}
    per_bit = collections.defaultdict(lambda: [0, 0, 0])  # planted, row flagged, corrected
    for k, b in planted.items():
        per_bit[b][0] += 1
        per_bit[b][1] += k[:3] in rows
        per_bit[b][2] += k in fixed
    return {
        "false_positive_rows": len(rows - planted_rows),
        "wrong_sites_corrected": len(fixed - set(planted)),
        "per_bit": {b: per_bit[b] for b in sorted(per_bit)},
    }


@pytest.mark.parametrize("csum", ["f64", "f32comp"])
def test_c3_campaign(csum, c3_oracle):
    """The whole 1000-sweep campaign twice: every seeded flip (the smallest detectable bit
    and the per-bit rates), and the flips outside the guard band against the oracle's run
    (events equal, grid within 1e-5), with the error against the fp64-storage oracle."""
    R = c3_oracle
    u0, C, plan = R["u0"], R["C"], R["plan"]
    say("C3 campaign", csum)
    g, ev, rep, shape = run_gpu(u0, W.THERMAL_TAPS, W.C3.nsweeps, C=C, eps=W.C3.eps, csum=csum,
                                plan=plan, max_events=1 << 16)
    s = _summary(plan, ev)
    s.update({"csum": csum, "corrected": rep["corrected"], "rows_flagged": rep["rows_flagged"],
              "checksum_faults": rep["checksum_faults"], "uncorrectable": rep["uncorrectable"],
              "max_noise": rep["max_noise"], "launch_shape": shape,
              "vs_fp64_oracle_all_flips": error_vs(g, R["ref64"])})
    assert rep["events_total"] < (1 << 16)
    assert s["false_positive_rows"] == 0 and s["wrong_sites_corrected"] == 0
    assert rep["uncorrectable"] == 0
    for b, (n, flagged, fixed) in s["per_bit"].items():
        if b >= B_MIN_GUARANTEED:
            assert flagged == n and fixed == n, (b, n, flagged, fixed)
        if b <= B_MAX_NEVER:
            assert flagged == 0, (b, flagged)

    kept, info = R["kept"], R["info"]
    say("C3 campaign oracle parity", csum, len(kept), "of", len(plan))
    g2, ev2, rep2, _ = run_gpu(u0, W.THERMAL_TAPS, W.C3.nsweeps, C=C, eps=W.C3.eps, csum=csum,
                               plan=kept, max_events=1 << 16)
    assert event_keys(ev2) == event_keys(R["events"])
    for k in ("rows_flagged", "corrected", "checksum_faults", "uncorrectable"):
        assert rep2[k] == R["counters"][k], k
    assert_grid_close(g2, R["grid"], 1e-5, f"C3 campaign {csum}")
    left = plan[info["skipped"] == 1]
    s.update({"oracle_parity_flips": int(len(kept)),
              "guard_band_left_out": {int(b): int(np.sum(left["bit"] == b))
                                      for b in np.unique(left["bit"])},
              "vs_fp64_oracle_parity_run": error_vs(g2, R["ref64"]),
              "oracle_vs_fp64_oracle": error_vs(R["grid"], R["ref64"])})
    write_summary(f"campaign_c3_{csum}.json", s)


@pytest.mark.parametrize("csum", ["f64", "f32comp"])
def test_c3_false_positives(csum, c3_oracle):
    """A fault-free 1000-sweep run: no row flagged in 32.8 million row tests, and the error of
    the fp32 grid against the fp64-storage oracle run stated."""
    nz, ny, nx = W.C3.shape
    u0, C = c3_oracle["u0"], c3_oracle["C"]
    say("C3 fault-free", csum)
    g, ev, rep, _ = run_gpu(u0, W.THERMAL_TAPS, W.C3.nsweeps, C=C, eps=W.C3.eps, csum=csum)
    write_summary(f"c3_fault_free_{csum}.json", {
        "csum": csum, "row_tests": nz * ny * W.C3.nsweeps, "false_positives": rep["rows_flagged"],
        "max_noise": rep["max_noise"], "vs_fp64_oracle": error_vs(g, c3_oracle["ref64"])})
    assert rep["rows_flagged"] == 0 and len(ev) == 0
    # the noise floor of an fp32 grid: a smooth row rounds alike, up to half an ulp of values
    # near 80 (2^-18 / 80 / 2 = 4.8e-8 relative) plus the earlier roundings of the chain
    assert rep["max_noise"] < 0.6 * W.C3.eps
