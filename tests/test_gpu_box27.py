"""27-point box stencils (every tap (dx, dy, dz) with offsets in -1..1) through the GPU path
against the oracle: bitwise where every operation is exact, every boundary rule with
asymmetric weights (x-boundary terms of nine rows per prediction), online location and
correction, offline rollback, and the 1024 x 1024 x 128 fp32 grid at full size.  Bars as for
the star stencils: fp64 grids within 1e-12, fp32 grids within 1e-5, events equal."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import assert_grid_close, event_keys, run_gpu, run_oracle, say

pytestmark = pytest.mark.gpu


def box27(wc, wface, wedge, wcorner, asym=1.0):
    """Taps by the number of non-zero offsets (0: centre, 1: face, 2: edge, 3: corner); asym
    scales every tap with dx = +1."""
    taps = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                n = abs(dx) + abs(dy) + abs(dz)
                w = (wc, wface, wedge, wcorner)[n] * (asym if dx == 1 else 1.0)
                taps.append((dx, dy, dz, w))
    return tuple(taps)


DYADIC27 = box27(0.25, 0.0625, 0.015625, 0.0078125)
SMOOTH27 = box27(0.4, 0.05, 0.015, 0.005)       # weights sum to 0.92
ASYM27 = box27(0.3, 0.06, 0.012, 0.004, asym=1.7)


# exact arithmetic: 2^-7 per sweep, values below 2^7 (5 sweeps fit fp64, 2 fit fp32)
@pytest.mark.parametrize("dtype,nsweeps", [(np.float64, 5), (np.float32, 2)])
@pytest.mark.parametrize("shape", [(6, 37, 64), (3, 20, 512), (4, 9, 7)])
@pytest.mark.parametrize("bc", ["clamp", "periodic"])
def test_box_dyadic_bitwise(dtype, nsweeps, shape, bc):
    rng = np.random.default_rng(29)
    u0 = rng.integers(0, 64, shape).astype(dtype)
    C = rng.integers(-4, 4, shape).astype(dtype)
    eps = 1e-12 if dtype == np.float64 else 1e-7
    say("box dyadic", dtype.__name__, shape, bc)
    g, gev, grep, _ = run_gpu(u0, DYADIC27, nsweeps, C=C, eps=eps, bc=bc)
    o, oev, ocnt = run_oracle(u0, DYADIC27, nsweeps, C=C, eps=eps, bc=bc)
    assert grep["rows_flagged"] == 0 and ocnt["rows_flagged"] == 0
    assert np.array_equal(g, o)


CASES = [
    ((5, 13, 9), np.float64, "clamp"),
    ((4, 17, 100), np.float32, "periodic"),
    ((3, 33, 252), np.float32, "constant"),
    ((6, 19, 260), np.float64, "constant"),
    ((2, 40, 96), np.float64, "periodic"),
    ((7, 70, 520), np.float32, "clamp"),
]


@pytest.mark.parametrize("shape,dtype,bc", CASES)
def test_box_online_boundaries(shape, dtype, bc):
    nz, ny, nx = shape
    rng = np.random.default_rng(nx * 11 + ny)
    u0 = (50 + 10 * rng.random(shape)).astype(dtype)
    C = rng.random(shape).astype(dtype)
    f64 = dtype == np.float64
    eps = 1e-12 if f64 else 1e-7 * max(1.0, (512.0 / min(nx, ny)) ** 0.5)
    bit = 60 if f64 else 28
    plan = W.make_plan([(3, nz // 2, ny - 1, nx - 1, bit), (6, 0, 1, 0, bit - 3)])
    say("box online", shape, dtype.__name__, bc)
    g, gev, grep, _ = run_gpu(u0, ASYM27, 9, C=C, eps=eps, bc=bc, bc_value=2.5, plan=plan)
    o, oev, ocnt = run_oracle(u0, ASYM27, 9, C=C, eps=eps, bc=bc, bc_value=2.5, plan=plan)
    assert event_keys(gev) == event_keys(oev)
    assert grep["corrected"] == 2
    assert_grid_close(g, o, 1e-12 if f64 else 1e-5, f"box {shape} {bc}")


@pytest.mark.parametrize("bc", ["clamp", "constant", "periodic"])
def test_box_offline(bc):
    shape = (6, 40, 96)
    rng = np.random.default_rng(9)
    u0 = 10 * rng.random(shape)
    plan = W.make_plan([(7, 1, 0, 95, 55), (13, 3, 39, 0, 62)])
    say("box offline", bc)
    g, gev, grep, _ = run_gpu(u0, ASYM27, 23, mode="offline", period=5, eps=1e-12, bc=bc,
                              bc_value=2.0, plan=plan)
    o, oev, ocnt = run_oracle(u0, ASYM27, 23, mode="offline", period=5, eps=1e-12, bc=bc,
                              bc_value=2.0, plan=plan)
    assert event_keys(gev) == event_keys(oev)
    assert grep["rollbacks"] == 2 and grep["windows_checked"] == ocnt["windows_checked"]
    assert np.array_equal(g, run_gpu(u0, ASYM27, 23, mode="none", bc=bc, bc_value=2.0)[0])
    assert_grid_close(g, o, 1e-12, "box offline")


def test_box_fp32_thermal_autotuned_graph():
    nz, ny, nx = 16, 96, 512
    u0, C = W.thermal_grid(nx, ny, nz, np.float32)
    plan = W.random_plan(79, 8, 40, (nz, ny, nx), list(range(16, 31)))
    say("box fp32, autotuned, graph")
    g, gev, grep, _ = run_gpu(u0, SMOOTH27, 40, C=C, eps=2e-7, plan=plan, autotune=True,
                              graph=True, chunks=[10] * 4)
    o, oev, ocnt = run_oracle(u0, SMOOTH27, 40, C=C, eps=2e-7, plan=plan)
    assert event_keys(gev) == event_keys(oev)
    assert grep["corrected"] == ocnt["corrected"] == len(plan)
    assert_grid_close(g, o, 1e-5, "box fp32 thermal")


def test_box_fullsize_parity():
    u0, C = W.C5.inputs()
    plan = W.make_plan([(2, 64, 512, 1023, 30), (7, 127, 0, 0, 27)])
    say("box full size")
    g, gev, grep, _ = run_gpu(u0, SMOOTH27, 10, C=C, eps=2e-7, plan=plan, autotune=True)
    o, oev, ocnt = run_oracle(u0, SMOOTH27, 10, C=C, eps=2e-7, plan=plan)
    assert event_keys(gev) == event_keys(oev)
    assert grep["corrected"] == 2
    assert_grid_close(g, o, 1e-5, "box full size")
