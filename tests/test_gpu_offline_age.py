"""Offline detection on the 1024 x 1024 x 128 fp32 thermal grid as a function of the flip's age
(sweeps between the flip and the window's comparison) and of the flipped bit: window k = 10,
threshold 1e-6, one flip per window, after 300 unprotected sweeps have brought the field close
to its steady state (values in [64, 128), row sums near 1024 * 80).

At age 0 a flip of mantissa bit b changes a value by 2^(b-17) and its row sum by the same, a
relative signal of about 2^(b-33.3): bits >= 14 exceed the threshold.  Each later sweep keeps
0.65 of the row's share of the error in the row (centre and x weights) and passes the rest to
the neighbouring rows and out through the ambient term, so the smallest detected bit rises
with the age.  Asserted: every flip of bit >= 20 is detected at every age, no flip of bit <= 10
is (its signal is below 1e-7 even at age 0), and the smallest bit detected at every site does
not fall by more than one as the age grows.  The measured table is written to
offline_bmin_vs_age.json in the results folder."""
import json
import os
import tempfile

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import say

pytestmark = pytest.mark.gpu
# where the run writes its result summary (JSON): $ABFT_TEST_OUT, else the system temp folder
OUT = os.environ.get("ABFT_TEST_OUT") or os.path.join(tempfile.gettempdir(), "abft_test_out")

K = 10
BITS = range(8, 25)
AGES = range(K)
REPS = 3
PRERUN = 300


def _plan(shape, first_window):
    nz, ny, nx = shape
    rng = np.random.default_rng(1006)
    rows, cells = [], []
    w = first_window
    for rep in range(REPS):
        for a in AGES:
            for b in BITS:
                t = w * K + (K - 1 - a)
                rows.append((t, int(rng.integers(0, nz)), int(rng.integers(0, ny)),
                             int(rng.integers(0, nx)), b))
                cells.append((w, a, b))
                w += 1
    return W.make_plan(rows), cells


def test_offline_bmin_vs_age():
    import torch
    from paper_1909_00709_amd import abft
    w5 = W.C5
    u0n, Cn = w5.inputs()
    stream = torch.cuda.Stream()
    say("offline b_min vs age: pre-run", PRERUN)
    with torch.cuda.stream(stream):
        C = torch.from_numpy(Cn).cuda()
        P = abft.Stencil(torch.from_numpy(u0n).cuda(), w5.taps, C=C, mode="none", stream=stream)
        P.step(PRERUN)
        start = P.current()[0].clone()
        P.close()
    plan, cells = _plan(w5.shape, 0)
    nwin = len(cells)
    say("offline b_min vs age:", nwin, "windows")
    with torch.cuda.stream(stream):
        S = abft.Stencil(start, w5.taps, C=C, mode="offline", period=K, threshold=w5.eps,
                         stream=stream, max_events=1 << 18)
        S.inject(plan)
        S.step(nwin * K)
        rep, ev = S.check()
        S.close()
    stream.synchronize()
    assert rep["events_total"] < (1 << 18)
    assert rep["persistent"] == 0
    rolled = {int(e["sweep"]) // K for e in ev if int(e["kind"]) == 6}
    det = {}
    for (w, a, b) in cells:
        det.setdefault((a, b), []).append(w in rolled)
    table = {a: {b: sum(det[(a, b)]) for b in BITS} for a in AGES}
    bmin = {}
    for a in AGES:
        full = [b for b in BITS if all(table[a][bb] == REPS for bb in BITS if bb >= b)]
        bmin[a] = min(full) if full else None
    summary = {"threshold": w5.eps, "period": K, "prerun_sweeps": PRERUN, "sites_per_cell": REPS,
               "detected": {str(a): {str(b): table[a][b] for b in BITS} for a in AGES},
               "bmin_all_sites": {str(a): bmin[a] for a in AGES},
               "windows_flagged": rep["windows_flagged"], "rollbacks": rep["rollbacks"],
               "max_noise": rep["max_noise"]}
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, "offline_bmin_vs_age.json"), "w") as f:
        json.dump(summary, f, indent=1)
    print(json.dumps({"bmin_all_sites": summary["bmin_all_sites"]}))
    for a in AGES:
        for b in BITS:
            if b >= 20:
                assert table[a][b] == REPS, (a, b, table[a])
            if b <= 10:
                assert table[a][b] == 0, (a, b, table[a])
    for a in range(1, K):
        assert bmin[a] is not None and bmin[a - 1] is not None
        assert bmin[a] >= bmin[a - 1] - 1, bmin
    # every rolled-back window holds a planted flip: no false positives
    assert rolled <= {c[0] for c in cells}
