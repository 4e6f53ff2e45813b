"""The paper's detectable-bit result on the GPU path (Section 5.3 with the parameters of Table 1):
64 x 64 x 8 fp32 tiles, 128 iterations, online detection with threshold 1e-5, one flip per run.
Flips of bits 13..31 are detected, located at their exact site and corrected; flips of bits
0..12 are not seen.  The 96 runs (32 bits x 3 sites) go through one batch, one grid per run,
with the same seeded flips as the oracle's pin of this result, and each grid's events are
compared with its oracle run."""
import json
import os

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import event_keys, run_oracle, say

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_paper_detectable_bits_gpu():
    import torch
    from paper_1909_00709_amd import abft
    with open(os.path.join(GOLDEN, "paper_table1_detection.json")) as f:
        fx = json.load(f)
    t = fx["tile"]
    nz, ny, nx = t["nz"], t["ny"], t["nx"]
    iters, eps = fx["iterations"], fx["detection_threshold"]
    u0, C = W.thermal_grid(nx, ny, nz, np.float32, t_amb=325.0)
    rng = np.random.default_rng(99)
    runs = []
    for bit in range(fx["word_bits"]):
        for rep in range(3):
            sweep = int(rng.integers(0, iters))
            runs.append((sweep, int(rng.integers(0, nz)), int(rng.integers(0, ny)),
                         int(rng.integers(0, nx)), bit))
    plan = W.empty_plan(len(runs))
    for g, r in enumerate(runs):
        for k, name in enumerate(("sweep", "z", "y", "x", "bit")):
            plan[g][name] = r[k]
        plan[g]["grid"] = g
    plan.sort(order="sweep", kind="stable")
    say("paper table 1 on the GPU:", len(runs), "grids")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        grids = [(torch.from_numpy(u0).cuda(), torch.from_numpy(C).cuda()) for _ in runs]
        B = abft.Batch(grids, W.THERMAL_TAPS, threshold=eps, stream=stream, max_events=1 << 14)
        B.inject(plan)
        B.step(iters)
        rep, ev = B.check()
        B.close()
    stream.synchronize()
    first, last = fx["detected_bits"]["first"], fx["detected_bits"]["last"]
    for g, r in enumerate(runs):
        gev = ev[ev["grid"] == g]
        detected = bool(np.any(gev["kind"] == 1))
        assert detected == (first <= r[4] <= last), (g, r)
        if detected:
            fixed = gev[gev["kind"] == 2]
            assert len(fixed) == 1 and tuple(int(fixed[0][f]) for f in
                                             ("sweep", "z", "y", "x")) == r[:4], (g, r)
        o, oev, ocnt = run_oracle(u0, W.THERMAL_TAPS, iters, C=C, eps=eps,
                                  plan=W.make_plan([r]))
        assert event_keys(gev) == event_keys(oev), (g, r)
    assert rep["uncorrectable"] == 0
