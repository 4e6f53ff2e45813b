"""Fault campaigns for the options on the 512 x 512 x 64 fp32 thermal grid, each against the
oracle: memory-resident flips with the input-side check (one per sweep, random sites, bits
18..30), store flips with tile-local checksums and the recompute correction (two per sweep in
different layers), and memory and store flips mixed with the recompute correction.

Bars: events equal to the oracle's; the final grid bitwise equal to the GPU's fault-free run
(every correction in these campaigns is exact) and within 1e-5 of the oracle."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import assert_grid_close, event_keys, run_gpu, run_oracle, say

pytestmark = pytest.mark.gpu

SHAPE = (64, 512, 512)
NSWEEPS = 40


def _inputs():
    nz, ny, nx = SHAPE
    return W.thermal_grid(nx, ny, nz, np.float32)


def _plan(seed, kinds, per_sweep, bits):
    rng = np.random.default_rng(seed)
    nz, ny, nx = SHAPE
    rows = []
    for t in range(2, NSWEEPS - 1):
        layers = rng.choice(nz, size=per_sweep, replace=False)
        for i, z in enumerate(layers):
            kind = kinds[(t + i) % len(kinds)]
            rows.append((t, int(z), int(rng.integers(0, ny)), int(rng.integers(0, nx)),
                         int(bits[int(rng.integers(0, len(bits)))]), 0, kind))
    return W.make_plan(rows)


@pytest.fixture(scope="module")
def clean():
    u0, C = _inputs()
    say("campaigns: fault-free run")
    return run_gpu(u0, W.THERMAL_TAPS, NSWEEPS, C=C, eps=1e-7, autotune=True)[0]


def _check(name, plan, clean, **kw):
    u0, C = _inputs()
    say("campaign:", name, len(plan), "flips")
    gkw = {k: v for k, v in kw.items() if k in ("correction", "tile_x", "input_check")}
    okw = {"recompute": kw.get("correction") == "recompute", "tile_x": kw.get("tile_x", 0),
           "input_check": kw.get("input_check", True)}
    eps = kw.get("eps", 1e-7)
    g, gev, grep, _ = run_gpu(u0, W.THERMAL_TAPS, NSWEEPS, C=C, eps=eps, plan=plan,
                              autotune=True, graph=True, chunks=[NSWEEPS // 4] * 4, **gkw)
    o, oev, ocnt = run_oracle(u0, W.THERMAL_TAPS, NSWEEPS, C=C, eps=eps, plan=plan, **okw)
    assert event_keys(gev) == event_keys(oev)
    assert grep["uncorrectable"] == 0 and grep["mem_unlocated"] == 0
    assert np.array_equal(g, clean), name
    assert_grid_close(g, o, 1e-5, name)
    return grep


def test_memory_flip_campaign(clean):
    plan = _plan(2001, [W.FAULT_MEMORY], 1, range(18, 31))
    rep = _check("memory flips", plan, clean)
    assert rep["mem_corrected"] == len(plan)


def test_tile_recompute_campaign(clean):
    plan = _plan(2002, [W.FAULT_STORE], 2, range(22, 31))
    rep = _check("tiles + recompute", plan, clean, tile_x=64, correction="recompute", eps=4e-7,
                 input_check=False)
    assert rep["corrected"] == len(plan)


def test_mixed_kinds_recompute_campaign(clean):
    plan = _plan(2003, [W.FAULT_MEMORY, W.FAULT_STORE], 2, range(20, 31))
    rep = _check("memory and store flips, recompute", plan, clean, correction="recompute")
    assert rep["mem_corrected"] + rep["corrected"] == len(plan)
