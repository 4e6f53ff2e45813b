"""The recompute correction through the GPU path: a located output point evaluated again from
the sweep's input (stencil locality) instead of being rebuilt from the checksums (Eq.(10)).

Bars: events equal to the oracle's (recompute mode); the final grid bitwise equal to the GPU's
own fault-free run (the recomputed value is the one the sweep stores for a clean input), for
fp32 and fp64, and within 1e-5 / 1e-12 of the oracle."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import assert_grid_close, event_keys, run_gpu, run_oracle, say
from tests.test_gpu_batch import _batch_plan, _run_batch
from tests.test_gpu_memory_faults import ASYM, BOX, STAR2

pytestmark = pytest.mark.gpu


def _thermal(shape, dtype=np.float32):
    nz, ny, nx = shape
    return W.thermal_grid(nx, ny, nz, dtype)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_recompute_thermal_bitwise(dtype):
    shape = (8, 48, 256)
    u0, C = _thermal(shape, dtype)
    f32 = dtype == np.float32
    eps = 1e-7 if f32 else 1e-12
    bits = list(range(22, 31)) if f32 else list(range(48, 62))
    plan = W.random_plan(91, 10, 20, shape, bits, distinct_sweeps=True)
    say("recompute correction, thermal", dtype.__name__)
    clean = run_gpu(u0, W.THERMAL_TAPS, 20, C=C, eps=eps)[0]
    g, gev, grep, _ = run_gpu(u0, W.THERMAL_TAPS, 20, C=C, eps=eps, plan=plan,
                              correction="recompute")
    o, oev, ocnt = run_oracle(u0, W.THERMAL_TAPS, 20, C=C, eps=eps, plan=plan, recompute=True)
    assert event_keys(gev) == event_keys(oev)
    assert grep["corrected"] == len(plan) == ocnt["corrected"]
    assert np.array_equal(g, clean)
    assert_grid_close(g, o, 1e-5 if f32 else 1e-12, "recompute")


def test_recompute_multiple_errors_in_a_layer():
    """Two and three flips in one layer on different rows and columns: uncorrectable with
    Eq.(10), corrected by evaluating every intersection again."""
    shape = (4, 64, 128)
    u0, C = _thermal(shape)
    plan = W.make_plan([(1, 1, 8, 21, 29), (1, 1, 30, 40, 28), (3, 2, 5, 5, 27),
                        (3, 2, 50, 100, 29), (3, 2, 60, 7, 30)])
    say("recompute, several errors per layer")
    clean = run_gpu(u0, W.THERMAL_TAPS, 5, C=C, eps=1e-7)[0]
    g, gev, grep, _ = run_gpu(u0, W.THERMAL_TAPS, 5, C=C, eps=1e-7, plan=plan,
                              correction="recompute")
    o, oev, ocnt = run_oracle(u0, W.THERMAL_TAPS, 5, C=C, eps=1e-7, plan=plan, recompute=True)
    assert event_keys(gev) == event_keys(oev)
    assert grep["uncorrectable"] == 0 and grep["corrected"] == 5
    assert np.array_equal(g, clean)
    e10 = run_gpu(u0, W.THERMAL_TAPS, 5, C=C, eps=1e-7, plan=plan)[2]
    assert e10["uncorrectable"] == 2


@pytest.mark.parametrize("taps", [ASYM, STAR2, BOX], ids=["star1", "star2", "box"])
@pytest.mark.parametrize("bc", ["clamp", "periodic", "constant"])
def test_recompute_stencils_and_boundaries(taps, bc):
    shape = (6, 20, 64)
    rng = np.random.default_rng(41)
    u0 = (20 + 5 * rng.random(shape)).astype(np.float32)
    C = rng.random(shape).astype(np.float32)
    plan = W.make_plan([(1, 0, 0, 0, 29), (3, 5, 19, 63, 28), (4, 2, 5, 11, 27),
                        (4, 2, 12, 3, 29)])
    kw = dict(C=C, eps=3e-7, bc=bc, bc_value=1.5)
    say("recompute", len(taps), "taps", bc)
    clean = run_gpu(u0, taps, 6, **kw)[0]
    g, gev, grep, _ = run_gpu(u0, taps, 6, plan=plan, correction="recompute", **kw)
    o, oev, _ = run_oracle(u0, taps, 6, plan=plan, recompute=True, **kw)
    assert event_keys(gev) == event_keys(oev)
    assert grep["corrected"] == 4 and grep["uncorrectable"] == 0
    assert np.array_equal(g, clean)


def test_recompute_graph_and_memory_faults_together():
    shape = (8, 32, 128)
    u0, C = _thermal(shape)
    plan = W.make_plan([(2, 3, 4, 5, 29), (5, 1, 30, 127, 28, 0, W.FAULT_MEMORY),
                        (9, 7, 0, 0, 30), (9, 7, 31, 64, 27)])
    say("recompute in graphs, with a memory flip")
    clean = run_gpu(u0, W.THERMAL_TAPS, 12, C=C, eps=1e-7)[0]
    g, gev, grep, _ = run_gpu(u0, W.THERMAL_TAPS, 12, C=C, eps=1e-7, plan=plan, graph=True,
                              chunks=[6, 6], correction="recompute")
    o, oev, _ = run_oracle(u0, W.THERMAL_TAPS, 12, C=C, eps=1e-7, plan=plan, recompute=True)
    assert event_keys(gev) == event_keys(oev)
    assert grep["corrected"] == 3 and grep["mem_corrected"] == 1
    assert np.array_equal(g, clean)


def test_recompute_batch():
    shapes = W.c4_shapes(10, seed=46)
    inputs = W.c4_inputs(shapes)
    per_grid = {0: W.make_plan([(2, 0, 1, 2, 29), (2, 0, 9, 30, 28)]),
                4: W.make_plan([(6, 1, 3, 3, 30)])}
    per_grid = {g: p for g, p in per_grid.items() if g < len(shapes)}
    plan = _batch_plan(per_grid)
    say("recompute in a batch")
    clean = _run_batch(shapes, inputs, 10, None)[0]
    outs, ev, rep, _ = _run_batch(shapes, inputs, 10, plan, correction="recompute")
    assert rep["corrected"] == 3 and rep["uncorrectable"] == 0
    for g in range(len(shapes)):
        assert np.array_equal(outs[g], clean[g]), g


def test_recompute_fullsize():
    u0, C = W.C5.inputs()
    plan = W.make_plan([(2, 64, 512, 1023, 30), (7, 127, 0, 0, 27), (7, 127, 900, 512, 29)])
    say("recompute, 1024 x 1024 x 128 fp32")
    clean = run_gpu(u0, W.THERMAL_TAPS, 10, C=C, eps=2e-7, autotune=True)[0]
    g, gev, grep, _ = run_gpu(u0, W.THERMAL_TAPS, 10, C=C, eps=2e-7, plan=plan, autotune=True,
                              correction="recompute")
    assert grep["corrected"] == 3 and grep["uncorrectable"] == 0
    assert np.array_equal(g, clean)
    o, oev, _ = run_oracle(u0, W.THERMAL_TAPS, 10, C=C, eps=2e-7, plan=plan, recompute=True)
    assert event_keys(gev) == event_keys(oev)
