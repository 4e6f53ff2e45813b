"""Memory-resident faults through the GPU path against the oracle: a bit flip of a sweep's
input grid after its checksums were taken and before the sweep reads it (the first case in
the proof of Theorem 2).  The protected sweep sums its input rows as it reads them and
compares them with the stored checksums; the locate/correct launch places the changed point
with the index-weighted row sums, restores it from the row checksum, evaluates again the
outputs that read it and tests the sweep's row flags again.

Bars: events equal to the oracle's; fp32 grids bitwise equal to the GPU's own fault-free run
(the restored value is exact and the outputs are evaluated with the sweep's operations) and
within 1e-5 of the oracle; fp64 grids within 1e-12 of the oracle."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import assert_grid_close, event_keys, run_gpu, run_oracle, say

pytestmark = pytest.mark.gpu

MEM = W.FAULT_MEMORY

ASYM = ((0, 0, 0, 0.3), (1, 0, 0, 0.25), (-1, 0, 0, 0.05), (0, 1, 0, 0.1), (0, -1, 0, 0.2),
        (0, 0, 1, 0.07), (0, 0, -1, 0.01))
STAR2 = ((0, 0, 0, 0.4), (1, 0, 0, 0.1), (-1, 0, 0, 0.08), (2, 0, 0, 0.02), (-2, 0, 0, 0.03),
         (0, 1, 0, 0.09), (0, -1, 0, 0.07), (0, 2, 0, 0.01), (0, -2, 0, 0.02), (0, 0, 1, 0.05),
         (0, 0, -1, 0.06), (0, 0, 2, 0.015), (0, 0, -2, 0.025))
BOX = tuple((dx, dy, dz, (0.3, 0.06, 0.012, 0.004)[abs(dx) + abs(dy) + abs(dz)] *
             (1.5 if dx == 1 else 1.0)) for dz in (-1, 0, 1) for dy in (-1, 0, 1)
            for dx in (-1, 0, 1))


def _thermal(shape, dtype=np.float32):
    nz, ny, nx = shape
    return W.thermal_grid(nx, ny, nz, dtype)


@pytest.mark.parametrize("bit", [18, 24, 29, 30])
def test_memory_flip_thermal(bit):
    shape = (8, 40, 256)
    u0, C = _thermal(shape)
    plan = W.make_plan([(3, 5, 17, 111, bit, 0, MEM)])
    say("memory flip, thermal fp32, bit", bit)
    clean = run_gpu(u0, W.THERMAL_TAPS, 8, C=C, eps=1e-7)[0]
    g, gev, grep, _ = run_gpu(u0, W.THERMAL_TAPS, 8, C=C, eps=1e-7, plan=plan)
    o, oev, ocnt = run_oracle(u0, W.THERMAL_TAPS, 8, C=C, eps=1e-7, plan=plan)
    assert event_keys(gev) == event_keys(oev)
    assert grep["mem_flagged"] == 1 and grep["mem_corrected"] == 1 and grep["corrected"] == 0
    assert np.array_equal(g, clean)
    assert_grid_close(g, o, 1e-5, "memory flip")


@pytest.mark.parametrize("taps", [ASYM, STAR2, BOX], ids=["star1", "star2", "box"])
@pytest.mark.parametrize("bc", ["clamp", "periodic", "constant"])
def test_memory_flip_stencils_and_boundaries(taps, bc):
    """Corner, row end and inner points in one run (different sweeps): windows that wrap or
    are cut, row-end values in the re-tested predictions."""
    shape = (6, 20, 64)
    rng = np.random.default_rng(37)
    u0 = (20 + 5 * rng.random(shape)).astype(np.float32)
    C = rng.random(shape).astype(np.float32)
    plan = W.make_plan([(1, 0, 0, 0, 28, 0, MEM), (3, 5, 19, 63, 29, 0, MEM),
                        (5, 2, 9, 1, 27, 0, MEM)])
    say("memory flips", len(taps), "taps", bc)
    kw = dict(C=C, eps=3e-7, bc=bc, bc_value=1.5)
    clean = run_gpu(u0, taps, 7, **kw)[0]
    g, gev, grep, _ = run_gpu(u0, taps, 7, plan=plan, **kw)
    o, oev, ocnt = run_oracle(u0, taps, 7, plan=plan, **kw)
    assert event_keys(gev) == event_keys(oev)
    assert grep["mem_corrected"] == 3 and grep["corrected"] == 0 and grep["uncorrectable"] == 0
    assert np.array_equal(g, clean)
    assert_grid_close(g, o, 1e-5, f"memory flips {bc}")


def test_memory_flip_fp64_and_compensated_fp32():
    shape = (4, 24, 96)
    u0, C = _thermal(shape, np.float64)
    plan = W.make_plan([(2, 3, 23, 95, 58, 0, MEM), (4, 0, 0, 0, 61, 0, MEM)])
    say("memory flips fp64")
    g, gev, grep, _ = run_gpu(u0, W.THERMAL_TAPS, 6, C=C, eps=1e-12, plan=plan)
    o, oev, ocnt = run_oracle(u0, W.THERMAL_TAPS, 6, C=C, eps=1e-12, plan=plan)
    assert event_keys(gev) == event_keys(oev) and grep["mem_corrected"] == 2
    assert_grid_close(g, o, 1e-12, "fp64")
    u0, C = _thermal(shape)
    plan = W.make_plan([(2, 3, 10, 40, 27, 0, MEM)])
    say("memory flip, compensated fp32 checksums")
    clean = run_gpu(u0, W.THERMAL_TAPS, 6, C=C, eps=1e-7, csum="f32comp")[0]
    g, gev, grep, _ = run_gpu(u0, W.THERMAL_TAPS, 6, C=C, eps=1e-7, csum="f32comp", plan=plan)
    o, oev, ocnt = run_oracle(u0, W.THERMAL_TAPS, 6, C=C, eps=1e-7, plan=plan)
    assert event_keys(gev) == event_keys(oev) and grep["mem_corrected"] == 1
    assert np.array_equal(g, clean)


def test_two_flips_one_row_and_mixed_kinds():
    shape = (6, 20, 64)
    u0, C = _thermal(shape)
    # two input flips in one row are not placed; a store flip in another layer of the same
    # sweep is located and corrected after the re-test
    plan = W.make_plan([(1, 1, 4, 3, 22, 0, MEM), (1, 1, 4, 20, 21, 0, MEM),
                        (3, 1, 5, 9, 29, 0, MEM), (3, 4, 14, 30, 28)])
    say("unplaced input flips and mixed kinds")
    g, gev, grep, _ = run_gpu(u0, W.THERMAL_TAPS, 5, C=C, eps=1e-7, plan=plan)
    o, oev, ocnt = run_oracle(u0, W.THERMAL_TAPS, 5, C=C, eps=1e-7, plan=plan)
    assert event_keys(gev) == event_keys(oev)
    assert grep["mem_unlocated"] == ocnt["mem_unlocated"] == 1
    assert grep["mem_corrected"] == 1 and grep["corrected"] == ocnt["corrected"]
    un_g = [e for e in gev if e["kind"] == 11][0]
    un_o = [e for e in oev if e["kind"] == 11][0]
    assert un_g["a"] == un_o["a"] and un_g["b"] == pytest.approx(un_o["b"], rel=1e-9)


def test_memory_flip_graph_and_manual_correct():
    shape = (8, 32, 128)
    u0, C = _thermal(shape)
    plan = W.make_plan([(4, 2, 7, 50, 29, 0, MEM), (13, 6, 31, 127, 26, 0, MEM)])
    say("memory flips in graphs")
    clean = run_gpu(u0, W.THERMAL_TAPS, 20, C=C, eps=1e-7)[0]
    g, gev, grep, _ = run_gpu(u0, W.THERMAL_TAPS, 20, C=C, eps=1e-7, plan=plan, graph=True,
                              chunks=[10, 10])
    o, oev, _ = run_oracle(u0, W.THERMAL_TAPS, 20, C=C, eps=1e-7, plan=plan)
    assert event_keys(gev) == event_keys(oev) and grep["mem_corrected"] == 2
    assert np.array_equal(g, clean)

    import torch
    from paper_1909_00709_amd import abft
    say("memory flip, detection only, then correct")
    ut = torch.from_numpy(u0).cuda()
    Ct = torch.from_numpy(C).cuda()
    S = abft.Stencil(ut, W.THERMAL_TAPS, C=Ct, threshold=1e-7, auto_correct=False)
    try:
        S.inject(W.make_plan([(2, 3, 11, 64, 29, 0, MEM)]))
        S.step(3)
        rep, ev = S.check()
        assert rep["mem_flagged"] == 1 and rep["pending"] >= 1
        st, rep, ev = S.correct()
        assert st == abft.ABFT_OK and rep["mem_corrected"] == 1
        cur, _ = S.current()
        ref = run_gpu(u0, W.THERMAL_TAPS, 3, C=C, eps=1e-7)[0]
        assert np.array_equal(cur.cpu().numpy(), ref)
    finally:
        S.close()


def test_offline_memory_flips():
    shape = (6, 24, 64)
    u0, C = _thermal(shape)
    inside = W.make_plan([(6, 1, 3, 30, 29, 0, MEM)])
    first = W.make_plan([(4, 1, 3, 30, 29, 0, MEM)])
    say("offline memory flips")
    clean = run_gpu(u0, W.THERMAL_TAPS, 12, C=C, mode="none")[0]
    kw = dict(C=C, mode="offline", period=4, eps=3e-7)
    g, gev, grep, _ = run_gpu(u0, W.THERMAL_TAPS, 12, plan=inside, **kw)
    o, oev, _ = run_oracle(u0, W.THERMAL_TAPS, 12, plan=inside, **kw)
    assert event_keys(gev) == event_keys(oev) and grep["rollbacks"] == 1
    assert np.array_equal(g, clean)
    g, gev, grep, _ = run_gpu(u0, W.THERMAL_TAPS, 12, plan=first, input_check=False, **kw)
    o, oev, _ = run_oracle(u0, W.THERMAL_TAPS, 12, plan=first, input_check=False, **kw)
    assert event_keys(gev) == event_keys(oev) and grep["persistent"] == 1
    none = run_gpu(u0, W.THERMAL_TAPS, 12, C=C, mode="none", plan=first)[0]
    assert np.array_equal(g, none)
    assert_grid_close(g, o, 1e-5, "offline first-input flip")


def test_memory_flip_fullsize():
    u0, C = W.C5.inputs()
    plan = W.make_plan([(2, 64, 512, 1023, 29, 0, MEM), (6, 0, 0, 0, 27, 0, MEM),
                        (7, 127, 1023, 500, 25)])
    say("memory flips, 1024 x 1024 x 128 fp32")
    g, gev, grep, _ = run_gpu(u0, W.THERMAL_TAPS, 10, C=C, eps=2e-7, plan=plan, autotune=True)
    o, oev, _ = run_oracle(u0, W.THERMAL_TAPS, 10, C=C, eps=2e-7, plan=plan)
    assert event_keys(gev) == event_keys(oev)
    assert grep["mem_corrected"] == 2 and grep["corrected"] == 1
    assert_grid_close(g, o, 1e-5, "full size")


def test_memory_faults_rejected_where_unsupported():
    import torch
    from paper_1909_00709_amd import abft
    S = abft.Stencil(torch.zeros((2, 8, 64), device="cuda"), W.THERMAL_TAPS)
    try:
        with pytest.raises(abft.AbftError):
            S.inject(W.make_plan([(0, 0, 0, 0, 3, 1, MEM)]))
    finally:
        S.close()


def test_memory_flip_without_input_check():
    """Input-side check off: the output check reports the reached rows as checksum-side
    mismatches, as the oracle does, and the grid follows the unprotected run."""
    shape = (6, 24, 128)
    u0, C = _thermal(shape)
    plan = W.make_plan([(3, 2, 7, 11, 29, 0, MEM)])
    say("memory flip, input check off")
    g, gev, grep, _ = run_gpu(u0, W.THERMAL_TAPS, 6, C=C, eps=1e-7, plan=plan,
                              input_check=False)
    o, oev, ocnt = run_oracle(u0, W.THERMAL_TAPS, 6, C=C, eps=1e-7, plan=plan,
                              input_check=False)
    assert event_keys(gev) == event_keys(oev)
    assert grep["mem_flagged"] == 0 and grep["checksum_faults"] == ocnt["checksum_faults"] > 0
    none = run_gpu(u0, W.THERMAL_TAPS, 6, C=C, mode="none", plan=plan)[0]
    assert np.array_equal(g, none)


def test_memory_flips_in_a_batch():
    """Batches: each grid's input rows checked and repaired in its own locate block; every
    grid against its own oracle run."""
    from tests.test_gpu_batch import _run_batch
    shapes = W.c4_shapes(10, seed=47)
    inputs = W.c4_inputs(shapes)
    per_grid = {0: W.make_plan([(2, 0, 1, 2, 29, 0, MEM)]),
                3: W.make_plan([(5, 1, 3, 3, 28, 0, MEM), (7, 2, 10, 40, 29)]),
                9: W.make_plan([(8, 0, 0, 0, 27, 0, MEM)])}
    rows = []
    for g, p in per_grid.items():
        for f in p:
            rows.append((int(f["sweep"]), int(f["z"]), int(f["y"]), int(f["x"]), int(f["bit"]),
                         0, int(f["kind"]), g))
    plan = W.empty_plan(len(rows))
    for i, r in enumerate(rows):
        for k, name in enumerate(("sweep", "z", "y", "x", "bit", "attempt", "kind", "grid")):
            plan[i][name] = r[k]
    plan.sort(order="sweep", kind="stable")
    say("memory flips in a batch")
    clean = _run_batch(shapes, inputs, 10, None)[0]
    outs, ev, rep, _ = _run_batch(shapes, inputs, 10, plan)
    assert rep["mem_corrected"] == 3 and rep["corrected"] == 1
    for g in range(len(shapes)):
        u0, C = inputs[g]
        o, oev, _ = run_oracle(u0, W.THERMAL_TAPS, 10, C=C, eps=1e-7, plan=per_grid.get(g))
        assert event_keys(ev[ev["grid"] == g]) == event_keys(oev), g
        if g in (0, 9):
            assert np.array_equal(outs[g], clean[g]), g
        assert_grid_close(outs[g], o, 1e-5, f"grid {g}")


@pytest.mark.parametrize("taps", [None, STAR2, BOX], ids=["thermal", "star2", "box"])
def test_offline_checkpoint_check(taps):
    """Offline with the input check: a flip of a window's first input (the checkpoint itself)
    is found before the rollback, restored, and the recompute gives the fault-free run."""
    shape = (6, 24, 64)
    if taps is None:
        u0, C = _thermal(shape)
        taps, eps = W.THERMAL_TAPS, 3e-7
    else:
        rng = np.random.default_rng(53)
        u0 = (20 + 5 * rng.random(shape)).astype(np.float32)
        C = rng.random(shape).astype(np.float32)
        eps = 1e-6
    first = W.make_plan([(4, 1, 3, 30, 29, 0, MEM), (8, 5, 23, 63, 28, 0, MEM)])
    kw = dict(C=C, mode="offline", period=4, eps=eps)
    say("offline checkpoint check", len(taps), "taps")
    clean = run_gpu(u0, taps, 12, C=C, mode="none")[0]
    g, gev, grep, _ = run_gpu(u0, taps, 12, plan=first, **kw)
    o, oev, ocnt = run_oracle(u0, taps, 12, plan=first, **kw)
    assert event_keys(gev) == event_keys(oev)
    assert grep["rollbacks"] == 2 and grep["persistent"] == 0 and grep["mem_corrected"] == 2
    assert np.array_equal(g, clean)
