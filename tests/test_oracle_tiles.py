"""Pins for the oracle's tile-local checksums: the method applied on sub-domains of T points
along x (Section 3.1 defines the sweep on a domain or sub-domain; the sections on detection
size the threshold by the domain, chunk or block the method is applied on, and the
experiments use tiles).  Pins: exact rational arithmetic for Theorem 1 on tiles, exact integer
tile sums, the reduction to the row scheme when a tile spans the row, and the cases the tiles
are for (two errors in one layer on different rows and columns, a change too small for a row
but not for a tile)."""
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from tests.test_oracle_pins import _exact_next, _random_taps


@pytest.mark.parametrize("seed", range(30))
def test_tile_theorem1_exact_rational(orc, seed):
    rng = np.random.default_rng(3000 + seed)
    T = int(rng.choice([2, 3, 4]))
    nz, ny = (int(v) for v in rng.integers(1, 5, 2))
    nx = T * int(rng.integers(1, 4))
    shape = (nz, ny, nx)
    bc = int(rng.integers(0, 3))
    radius = int(rng.integers(1, 3))
    taps = []
    for dx, dy, dz, _ in _random_taps(rng, radius, int(rng.integers(1, 8))):
        if abs(dx) <= min(nx, T) and abs(dy) <= ny and abs(dz) <= nz:
            taps.append((dx, dy, dz, int(rng.integers(-8, 9)) / 8.0))
    g = int(rng.integers(-4, 5)) / 2.0
    ui = rng.integers(-64, 64, shape)
    Ci = rng.integers(-16, 16, shape)
    uF = [[[Fraction(int(v)) for v in row] for row in lay] for lay in ui]
    CF = [[[Fraction(int(v)) for v in row] for row in lay] for lay in Ci]
    nxt = _exact_next(uF, CF, [(dx, dy, dz, Fraction(w)) for dx, dy, dz, w in taps], bc,
                      Fraction(g))
    exact = np.array([[[float(sum(nxt[z][y][k * T:(k + 1) * T])) for k in range(nx // T)]
                       for y in range(ny)] for z in range(nz)])
    p = orc.Problem(shape, orc.F64, taps, bc=bc, bc_value=g)
    u, C = ui.astype(np.float64), Ci.astype(np.float64)
    pred = p.predict_tiles(p.const_tile_checksums(C, T), p.tile_checksums(u, T), u, T)
    assert np.array_equal(pred, exact)


def test_tile_sums_exact_and_whole_row_tile(orc):
    rng = np.random.default_rng(6)
    u = rng.integers(-1000, 1000, (3, 5, 48)).astype(np.float64)
    p = orc.Problem(u.shape, orc.F64, W.THERMAL_TAPS)
    for T in (1, 4, 16, 48):
        ref = u.astype(np.int64).reshape(3, 5, 48 // T, T).sum(axis=3)
        assert np.array_equal(p.tile_checksums(u, T), ref.astype(np.float64))
    # a tile that spans the row is the row checksum, and its prediction the row prediction
    C = rng.integers(-5, 5, u.shape).astype(np.float64)
    for bc in (0, 1, 2):
        q = orc.Problem(u.shape, orc.F64, [(0, 0, 0, 0.5), (1, 0, 0, 0.25), (-1, 0, 0, 0.125),
                                           (0, 1, 0, 0.0625), (0, 0, -1, 0.0625)], bc=bc,
                        bc_value=2.0)
        whole = q.predict_tiles(q.const_tile_checksums(C, 48), q.tile_checksums(u, 48), u, 48)
        assert np.array_equal(whole[..., 0], q.predict_rows_from_grid(u, C))


def _thermal(shape, dtype=np.float32):
    nz, ny, nx = shape
    return W.thermal_grid(nx, ny, nz, dtype)


def test_tiles_fault_free_and_single_flips(orc):
    shape = (4, 24, 128)
    u0, C = _thermal(shape)
    p = orc.Problem(shape, orc.F32, W.THERMAL_TAPS)
    clean, ev, cnt = p.run(u0, 10, C, eps=4e-7, tile_x=64)
    assert cnt["rows_flagged"] == 0
    plan = W.make_plan([(2, 1, 5, 70, 29), (6, 3, 23, 127, 27), (8, 0, 0, 0, 30)])
    fin, ev, cnt = p.run(u0, 10, C, eps=4e-7, tile_x=64, faults=plan)
    assert cnt["corrected"] == 3 and cnt["uncorrectable"] == 0
    flags = ev[ev["kind"] == orc.EV_ROW_FLAG]
    # each flip is seen by the tile that holds it (x = the tile's first point)
    assert {(int(e["sweep"]), int(e["z"]), int(e["y"]), int(e["x"])) for e in flags} == \
        {(2, 1, 5, 64), (6, 3, 23, 64), (8, 0, 0, 0)}
    np.testing.assert_allclose(fin, clean, rtol=1e-5)
    rec, _, cnt = p.run(u0, 10, C, eps=4e-7, tile_x=64, faults=plan, recompute=True)
    assert cnt["corrected"] == 3 and np.array_equal(rec, clean)


def test_tiles_separate_two_errors_in_a_layer(orc):
    """Two flips in one layer on different rows and columns: two rows and two columns for the
    row scheme (uncorrectable with Eq.(10)); in different tiles each flagged tile holds one
    flagged column, and both are corrected."""
    shape = (2, 32, 128)
    u0, C = _thermal(shape)
    p = orc.Problem(shape, orc.F32, W.THERMAL_TAPS)
    clean, _, _ = p.run(u0, 3, C, eps=4e-7)
    plan = W.make_plan([(1, 1, 4, 10, 28), (1, 1, 20, 100, 29)])
    _, _, rows = p.run(u0, 3, C, eps=4e-7, faults=plan)
    assert rows["uncorrectable"] == 1
    fin, ev, cnt = p.run(u0, 3, C, eps=4e-7, tile_x=64, faults=plan)
    assert cnt["uncorrectable"] == 0 and cnt["corrected"] == 2
    np.testing.assert_allclose(fin, clean, rtol=1e-5)
    # the same pair inside one tile's x range is ambiguous for Eq.(10) on tiles as well
    same = W.make_plan([(1, 1, 4, 10, 28), (1, 1, 20, 40, 29)])
    _, _, cnt = p.run(u0, 3, C, eps=4e-7, tile_x=64, faults=same)
    assert cnt["uncorrectable"] == 1
    fin, _, cnt = p.run(u0, 3, C, eps=4e-7, tile_x=64, faults=same, recompute=True)
    assert cnt["corrected"] == 2 and np.array_equal(fin, clean)


def test_tiles_are_more_sensitive(orc):
    """A change of 2^-3 relative to a value is about 1.2e-4 of a 1024-point row sum and 2e-3
    of a 64-point tile sum: below a 5e-4 threshold for the row, above it for the tile."""
    shape = (1, 8, 1024)
    u0, C = _thermal(shape)
    p = orc.Problem(shape, orc.F32, W.THERMAL_TAPS)
    plan = W.make_plan([(1, 0, 3, 500, 20)])  # mantissa bit 20 of a value in [256, 512)
    _, _, rows = p.run(u0, 2, C, eps=5e-4, faults=plan)
    assert rows["rows_flagged"] == 0
    _, _, tiles = p.run(u0, 2, C, eps=5e-4, tile_x=64, faults=plan)
    assert tiles["rows_flagged"] == 1 and tiles["corrected"] == 1


def test_tile_checksum_side_fault(orc):
    """Short tiles, long columns: a flip seen by its tile but not by its column is reported as
    a checksum-side mismatch of that tile, and the grid is left alone."""
    shape = (1, 512, 8)
    u0 = np.full(shape, 100.0, np.float32) + np.random.default_rng(1).random(shape).astype(
        np.float32)
    p = orc.Problem(shape, orc.F32, W.JACOBI_TAPS)
    plan = W.make_plan([(0, 0, 100, 6, 16)])
    fin, ev, cnt = p.run(u0, 1, eps=2e-5, tile_x=4, faults=plan)
    assert cnt["rows_flagged"] == 1 and cnt["cols_flagged"] == 0
    assert cnt["checksum_faults"] == 1 and cnt["corrected"] == 0
    e = ev[ev["kind"] == orc.EV_CHECKSUM_FAULT][0]
    assert (e["y"], e["x"]) == (100, 4)


def test_tile_mode_rejected_where_undefined(orc):
    p = orc.Problem((2, 4, 12), orc.F32, W.THERMAL_TAPS)
    u = np.zeros((2, 4, 12), np.float32)
    with pytest.raises(ValueError):
        p.run(u, 1, tile_x=5)  # does not divide nx
    with pytest.raises(ValueError):
        p.run(u, 1, mode=orc.MODE_OFFLINE, tile_x=4)
