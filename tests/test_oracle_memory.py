"""Pins for the oracle's memory-resident fault model: a bit flip of a sweep's input grid after
its checksums were taken and before the sweep reads it (the first case in the proof of
Theorem 2: the direct checksums of the next sweep are wrong, the interpolated ones right).

Online, the oracle compares the sums of the input rows as read with the stored checksums,
places the changed point with the index-weighted row sums W = sum_x (x + 1) u, recovers its
value from the row checksum, evaluates again the outputs that read it, and tests the sweep's
row flags again.  The pins come from outside the repair: the run without faults, the run with
the flip applied by hand between sweeps, exact integer sums, and the set of rows a changed
input can reach through the stencil.
"""
import numpy as np
import pytest

import workloads as W

MEM = W.FAULT_MEMORY


def _flip(v, bit):
    a = np.array([v])
    u = a.view(np.uint32 if a.dtype == np.float32 else np.uint64)
    u ^= type(u[0])(1) << type(u[0])(bit)
    return a[0]


def _thermal(shape, dtype=np.float32):
    nz, ny, nx = shape
    return W.thermal_grid(nx, ny, nz, dtype)


def test_weighted_row_sums_exact(orc):
    """Integer data: W equals the exact integer sum of (x + 1) u."""
    rng = np.random.default_rng(4)
    u = rng.integers(-1000, 1000, (3, 5, 37)).astype(np.float64)
    p = orc.Problem(u.shape, orc.F64, W.THERMAL_TAPS)
    ref = (u.astype(np.int64) * np.arange(1, 38, dtype=np.int64)).sum(axis=2)
    assert np.array_equal(p.weighted_row_checksums(u), ref.astype(np.float64))


def test_memory_flip_matches_manual_flip_unprotected(orc):
    """Kind MEMORY on sweep t hits u^t: the unprotected run equals t clean sweeps, the flip
    applied by hand, and the remaining sweeps."""
    shape = (4, 12, 40)
    u0, C = _thermal(shape)
    p = orc.Problem(shape, orc.F32, W.THERMAL_TAPS)
    t, z, y, x, bit = 3, 2, 7, 11, 27
    plan = W.make_plan([(t, z, y, x, bit, 0, MEM)])
    got, _, _ = p.run(u0, 8, C, mode=orc.MODE_NONE, faults=plan)
    ut, _, _ = p.run(u0, t, C, mode=orc.MODE_NONE)
    ut = ut.copy()
    ut[z, y, x] = _flip(ut[z, y, x], bit)
    ref, _, _ = p.run(ut, 8 - t, C, mode=orc.MODE_NONE)
    assert np.array_equal(got, ref)
    clean, _, _ = p.run(u0, 8, C, mode=orc.MODE_NONE)
    assert not np.array_equal(got, clean)


@pytest.mark.parametrize("bit", [18, 24, 29, 30])
def test_memory_flip_repaired_bitwise_fp32(orc, bit):
    """One input flip: one input row flagged, the point placed and restored exactly, the run
    equal to the fault-free run bitwise; the sweep's own flags lie in the rows the changed
    point reaches and are all cleared by the repair (no output point is corrected)."""
    shape = (4, 12, 40)
    u0, C = _thermal(shape)
    p = orc.Problem(shape, orc.F32, W.THERMAL_TAPS)
    clean, _, _ = p.run(u0, 8, C, eps=1e-7)
    t, z, y, x = 3, 2, 7, 11
    plan = W.make_plan([(t, z, y, x, bit, 0, MEM)])
    fin, ev, cnt = p.run(u0, 8, C, eps=1e-7, faults=plan)
    assert np.array_equal(fin, clean)
    assert cnt["mem_flagged"] == 1 and cnt["mem_corrected"] == 1 and cnt["mem_unlocated"] == 0
    assert cnt["corrected"] == 0 and cnt["cols_flagged"] == 0 and cnt["uncorrectable"] == 0
    mf = ev[ev["kind"] == orc.EV_MEM_FLAG]
    assert (mf["sweep"][0], mf["z"][0], mf["y"][0]) == (t, z, y)
    mc = ev[ev["kind"] == orc.EV_MEM_CORRECTED][0]
    ut, _, _ = p.run(u0, t, C, mode=orc.MODE_NONE)
    assert (mc["sweep"], mc["z"], mc["y"], mc["x"]) == (t, z, y, x)
    assert mc["b"] == ut[z, y, x] and mc["a"] == _flip(ut[z, y, x], bit)
    reach = {(z, y), (z, y - 1), (z, y + 1), (z - 1, y), (z + 1, y)}
    rows = {(int(e["z"]), int(e["y"])) for e in ev[ev["kind"] == orc.EV_ROW_FLAG]}
    assert rows <= reach and all(e["sweep"] == t for e in ev[ev["kind"] == orc.EV_ROW_FLAG])
    if bit >= 24:
        assert (z, y) in rows


def test_memory_flip_without_repair(orc):
    """Detection only: the input row and the reached rows are reported, the grid is not
    repaired."""
    shape = (4, 12, 40)
    u0, C = _thermal(shape)
    p = orc.Problem(shape, orc.F32, W.THERMAL_TAPS)
    clean, _, _ = p.run(u0, 6, C, eps=1e-7)
    plan = W.make_plan([(2, 1, 5, 20, 29, 0, MEM)])
    fin, ev, cnt = p.run(u0, 6, C, eps=1e-7, auto_correct=False, faults=plan)
    assert cnt["mem_flagged"] == 1 and cnt["mem_corrected"] == 0 and cnt["rows_flagged"] >= 1
    assert not np.array_equal(fin, clean)


def test_two_flips_in_one_row_unlocated(orc):
    """Two changes in one input row move W by a weighted mean of their positions, which the
    position test rejects; nothing in the input is changed by the repair step."""
    shape = (2, 10, 32)
    u0, C = _thermal(shape)
    p = orc.Problem(shape, orc.F32, W.THERMAL_TAPS)
    # values in [256, 512): bits 22 and 21 are worth 128 and 64, so both changes are exact
    plan = W.make_plan([(1, 1, 4, 3, 22, 0, MEM), (1, 1, 4, 20, 21, 0, MEM)])
    _, ev, cnt = p.run(u0, 3, C, eps=1e-7, faults=plan)
    assert cnt["mem_flagged"] == 1 and cnt["mem_unlocated"] == 1 and cnt["mem_corrected"] == 0
    un = ev[ev["kind"] == orc.EV_MEM_UNLOCATED][0]
    assert (un["sweep"], un["z"], un["y"]) == (1, 1, 4)
    u1, _, _ = p.run(u0, 1, C, mode=orc.MODE_NONE)
    d1 = float(_flip(u1[1, 4, 3], 22)) - float(u1[1, 4, 3])
    d2 = float(_flip(u1[1, 4, 20], 21)) - float(u1[1, 4, 20])
    assert un["a"] == d1 + d2
    assert un["b"] == pytest.approx((4 * d1 + 21 * d2) / (d1 + d2), rel=1e-12)


ASYM = [(0, 0, 0, 0.3), (1, 0, 0, 0.25), (-1, 0, 0, 0.05), (0, 1, 0, 0.1), (0, -1, 0, 0.2),
        (0, 0, 1, 0.07), (0, 0, -1, 0.01)]
STAR2 = [(0, 0, 0, 0.4), (1, 0, 0, 0.1), (-1, 0, 0, 0.08), (2, 0, 0, 0.02), (-2, 0, 0, 0.03),
         (0, 1, 0, 0.09), (0, -1, 0, 0.07), (0, 2, 0, 0.01), (0, -2, 0, 0.02), (0, 0, 1, 0.05),
         (0, 0, -1, 0.06), (0, 0, 2, 0.015), (0, 0, -2, 0.025)]
BOX = [(dx, dy, dz, (0.3, 0.06, 0.012, 0.004)[abs(dx) + abs(dy) + abs(dz)] * (1.5 if dx == 1
       else 1.0)) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


@pytest.mark.parametrize("taps", [ASYM, STAR2, BOX], ids=["star1", "star2", "box"])
@pytest.mark.parametrize("bc", [0, 1, 2])
@pytest.mark.parametrize("where", ["corner", "edge", "inner"])
def test_memory_repair_all_stencils_and_boundaries(orc, taps, bc, where):
    """Corners and row ends: the window of outputs to evaluate again wraps (periodic) or is cut
    (clamp, constant), and the row-end values enter the x-boundary terms of the predictions
    tested again.  fp32 data: the run equals the fault-free run bitwise."""
    shape = (5, 9, 24)
    rng = np.random.default_rng(31)
    u0 = (20 + 5 * rng.random(shape)).astype(np.float32)
    C = rng.random(shape).astype(np.float32)
    p = orc.Problem(shape, orc.F32, taps, bc=bc, bc_value=1.5)
    pos = {"corner": (0, 0, 0), "edge": (4, 8, 23), "inner": (2, 4, 1)}[where]
    plan = W.make_plan([(2, *pos, 28, 0, MEM)])
    clean, _, _ = p.run(u0, 5, C, eps=3e-7)
    fin, ev, cnt = p.run(u0, 5, C, eps=3e-7, faults=plan)
    assert cnt["mem_corrected"] == 1 and cnt["corrected"] == 0 and cnt["uncorrectable"] == 0
    assert np.array_equal(fin, clean)


def test_memory_repair_fp64_within_rounding(orc):
    shape = (4, 16, 48)
    u0, C = _thermal(shape, np.float64)
    p = orc.Problem(shape, orc.F64, W.THERMAL_TAPS)
    clean, _, _ = p.run(u0, 6, C, eps=1e-12)
    plan = W.make_plan([(2, 3, 15, 47, 58, 0, MEM), (4, 0, 0, 0, 61, 0, MEM)])
    fin, ev, cnt = p.run(u0, 6, C, eps=1e-12, faults=plan)
    assert cnt["mem_corrected"] == 2 and cnt["corrected"] == 0
    np.testing.assert_allclose(fin, clean, rtol=1e-12, atol=0)


def test_memory_and_store_flips_in_one_sweep(orc):
    """A memory flip and a store flip in different layers of one sweep: the memory repair
    clears the rows it explains, the store flip is then located and corrected as usual."""
    shape = (6, 20, 40)
    u0, C = _thermal(shape)
    p = orc.Problem(shape, orc.F32, W.THERMAL_TAPS)
    clean, _, _ = p.run(u0, 5, C, eps=1e-7)
    plan = W.make_plan([(2, 1, 5, 9, 29, 0, MEM), (2, 4, 14, 30, 28)])
    fin, ev, cnt = p.run(u0, 5, C, eps=1e-7, faults=plan)
    assert cnt["mem_corrected"] == 1 and cnt["corrected"] == 1
    np.testing.assert_allclose(fin, clean, rtol=1e-5)


def test_offline_memory_flip(orc):
    """Offline: a flip inside a window is undone by the rollback.  A flip of a window's first
    input hits the checkpoint as well: without the input check the recompute repeats it and the
    window stays flagged (persistent), the run equal to the unprotected run with that flip; with
    it, the checkpoint's rows are checked against their stored checksums before the rollback,
    the point is restored, and the run equals the fault-free run."""
    shape = (4, 16, 32)
    u0, C = _thermal(shape)
    p = orc.Problem(shape, orc.F32, W.THERMAL_TAPS)
    clean, _, _ = p.run(u0, 12, C, mode=orc.MODE_NONE)
    kw = dict(mode=orc.MODE_OFFLINE, period=4, eps=3e-7)
    inside = W.make_plan([(6, 1, 3, 30, 29, 0, MEM)])
    fin, ev, cnt = p.run(u0, 12, C, faults=inside, **kw)
    assert cnt["rollbacks"] == 1 and cnt["persistent"] == 0 and cnt["mem_flagged"] == 0
    assert np.array_equal(fin, clean)
    first = W.make_plan([(4, 1, 3, 30, 29, 0, MEM)])
    fin, ev, cnt = p.run(u0, 12, C, faults=first, input_check=False, **kw)
    assert cnt["rollbacks"] == 1 and cnt["persistent"] == 1
    none, _, _ = p.run(u0, 12, C, mode=orc.MODE_NONE, faults=first)
    assert np.array_equal(fin, none)
    fin, ev, cnt = p.run(u0, 12, C, faults=first, **kw)
    assert cnt["rollbacks"] == 1 and cnt["persistent"] == 0
    assert cnt["mem_flagged"] == 1 and cnt["mem_corrected"] == 1
    mc = ev[ev["kind"] == orc.EV_MEM_CORRECTED][0]
    assert (mc["sweep"], mc["z"], mc["y"], mc["x"]) == (4, 1, 3, 30)
    assert np.array_equal(fin, clean)


def test_bad_fault_kind_rejected(orc):
    shape = (2, 4, 8)
    p = orc.Problem(shape, orc.F32, W.THERMAL_TAPS)
    plan = W.make_plan([(0, 0, 0, 0, 3, 0, 2)])
    with pytest.raises(ValueError):
        p.run(np.zeros(shape, np.float32), 1, faults=plan)


def test_memory_flip_without_input_check(orc):
    """With the input-side check off, the output check still sees the flip one sweep later
    (Theorem 2: the direct checksums are wrong, the predicted ones right), in the rows the
    changed point reaches, but nothing places it: the layer's columns agree with their
    prediction from the changed input, so the mismatches are reported as checksum-side."""
    shape = (4, 12, 40)
    u0, C = _thermal(shape)
    p = orc.Problem(shape, orc.F32, W.THERMAL_TAPS)
    t, z, y, x = 3, 2, 7, 11
    plan = W.make_plan([(t, z, y, x, 29, 0, MEM)])
    fin, ev, cnt = p.run(u0, 6, C, eps=1e-7, faults=plan, input_check=False)
    assert cnt["mem_flagged"] == 0 and cnt["mem_corrected"] == 0
    rows = {(int(e["z"]), int(e["y"])) for e in ev[ev["kind"] == orc.EV_ROW_FLAG]}
    assert (z, y) in rows and rows <= {(z, y), (z, y - 1), (z, y + 1), (z - 1, y), (z + 1, y)}
    assert cnt["corrected"] == 0 and cnt["checksum_faults"] == len(rows)
    none, _, _ = p.run(u0, 6, C, mode=orc.MODE_NONE, faults=plan)
    assert np.array_equal(fin, none)
