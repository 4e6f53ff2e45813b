"""The offline rollback recompute (one launch, grid barriers between the window's sweeps):
persistent faults, partial windows, several tiles per block, and the shortest and longest
windows, each against the oracle and, where the rollback erases the flip, against the
fault-free run bitwise."""
import os
import tempfile

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import assert_grid_close, event_keys, run_gpu, run_oracle, say

pytestmark = pytest.mark.gpu


def test_persistent_fault():
    """A flip that recurs in the recompute (attempt 1): the re-check flags the window again
    and a persistent-fault event is reported, as in the oracle."""
    nz, ny, nx = 4, 64, 128
    u0, C = W.thermal_grid(nx, ny, nz, np.float64)
    plan = W.make_plan([(7, 1, 10, 20, 60, 0), (7, 1, 10, 20, 60, 1)])
    say("offline persistent")
    g, gev, grep, _ = run_gpu(u0, W.THERMAL_TAPS, 15, C=C, mode="offline", period=5,
                              eps=1e-12, plan=plan)
    o, oev, ocnt = run_oracle(u0, W.THERMAL_TAPS, 15, C=C, mode="offline", period=5, eps=1e-12,
                              plan=plan)
    assert event_keys(gev) == event_keys(oev)
    assert grep["persistent"] == ocnt["persistent"] == 1
    assert grep["rollbacks"] == 1
    assert_grid_close(g, o, 1e-12, "persistent")


def test_partial_window_rollback():
    """25 sweeps with period 10: the flip lies in the partial window (sweeps 20..24), which the
    check closes; its 5-sweep recompute erases it."""
    nz, ny, nx = 8, 96, 256
    u0, C = W.thermal_grid(nx, ny, nz, np.float32)
    plan = W.make_plan([(22, 5, 50, 100, 29)])
    say("offline partial window")
    g, gev, grep, _ = run_gpu(u0, W.THERMAL_TAPS, 25, C=C, mode="offline", period=10,
                              eps=W.C5.eps, plan=plan)
    o, oev, ocnt = run_oracle(u0, W.THERMAL_TAPS, 25, C=C, mode="offline", period=10,
                              eps=W.C5.eps, plan=plan)
    assert event_keys(gev) == event_keys(oev)
    assert grep["rollbacks"] == 1 and grep["windows_checked"] == ocnt["windows_checked"]
    clean = run_gpu(u0, W.THERMAL_TAPS, 25, C=C, mode="none")[0]
    assert np.array_equal(g, clean)


@pytest.mark.parametrize("nw", [4, 8])
def test_several_tiles_per_block(nw):
    """One plane per tile: 1024 or 2048 tiles, more than one wave of blocks, so every block of
    the recompute takes several tiles of each sweep."""
    import torch
    from paper_1909_00709_amd import abft
    nz, ny, nx = 32, 256, 256
    u0, C = W.thermal_grid(nx, ny, nz, np.float32)
    plan = W.make_plan([(3, 7, 200, 13, 28), (16, 30, 1, 255, 30)])
    fd, cache = tempfile.mkstemp(suffix=".tune")
    os.close(fd)
    try:
        with open(cache, "w") as f:  # dtype nx ny nz mode csum lpr nch vec tz pf nw
            f.write(f"{W.F32} {nx} {ny} {nz} {abft.ABFT_MODE_OFFLINE} 0 64 1 4 1 1 {nw}\n")
        say("offline recompute, tz 1, nw", nw)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            S = abft.Stencil(torch.from_numpy(u0).cuda(), W.THERMAL_TAPS,
                             C=torch.from_numpy(C).cuda(), mode="offline", period=10,
                             threshold=W.C5.eps, stream=stream, tuning_cache=cache,
                             input_check=False)
            rows, planes, lanes = S.launch_shape()
            assert (rows, planes, lanes) == (nw, 1, 64)
            S.inject(plan)
            S.step(20)
            rep, ev = S.check()
            g = S.current()[0].cpu().numpy()
            S.close()
        stream.synchronize()
    finally:
        os.unlink(cache)
    o, oev, ocnt = run_oracle(u0, W.THERMAL_TAPS, 20, C=C, mode="offline", period=10,
                              eps=W.C5.eps, plan=plan)
    assert event_keys(ev) == event_keys(oev)
    assert rep["rollbacks"] == 2
    clean = run_gpu(u0, W.THERMAL_TAPS, 20, C=C, mode="none")[0]
    assert np.array_equal(g, clean)


@pytest.mark.parametrize("period", [1, 2, 32, 128])
def test_window_lengths(period):
    """The shortest windows (no barrier, one barrier) and long ones (checked in chunks of 16
    interpolation steps; 127 barriers in the longest recompute)."""
    nz, ny, nx = 8, 32, 128
    u0, C = W.thermal_grid(nx, ny, nz, np.float64)
    nsweeps = 2 * period + 1
    plan = W.make_plan([(period // 2, 3, 17, 64, 57), (period + period // 2, 6, 2, 5, 61)])
    say("offline window length", period)
    g, gev, grep, _ = run_gpu(u0, W.THERMAL_TAPS, nsweeps, C=C, mode="offline", period=period,
                              eps=1e-12, plan=plan)
    o, oev, ocnt = run_oracle(u0, W.THERMAL_TAPS, nsweeps, C=C, mode="offline",
                              period=period, eps=1e-12, plan=plan)
    assert event_keys(gev) == event_keys(oev)
    assert grep["rollbacks"] == 2
    clean = run_gpu(u0, W.THERMAL_TAPS, nsweeps, C=C, mode="none")[0]
    assert np.array_equal(g, clean)
