"""Pins for the oracle's recompute correction (stencil locality): online, the sweep's input is
intact when a mismatch is found, so a located output point can be evaluated again from its
stencil neighbours instead of being rebuilt from the checksums (Eq.(10)).  The pins come from
outside the correction: the fault-free run, and the case analysis of Section 3.5 (one error per
flagged row or column, several rows and columns flagged together)."""
import numpy as np
import pytest

import workloads as W


def _thermal(shape, dtype=np.float32):
    nz, ny, nx = shape
    return W.thermal_grid(nx, ny, nz, dtype)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_single_flips_restored_bitwise(orc, dtype):
    """Each flip is put back to the exact fault-free value, so the whole run equals the
    fault-free run bitwise (fp32 and fp64), where Eq.(10) is only within rounding."""
    shape = (6, 24, 48)
    u0, C = _thermal(shape, dtype)
    code = orc.F32 if dtype == np.float32 else orc.F64
    eps = 1e-7 if dtype == np.float32 else 1e-12
    p = orc.Problem(shape, code, W.THERMAL_TAPS)
    clean, _, _ = p.run(u0, 12, C, eps=eps)
    bits = range(22, 31) if dtype == np.float32 else range(48, 62)
    plan = W.random_plan(77, 8, 12, shape, list(bits), distinct_sweeps=True)
    fin, ev, cnt = p.run(u0, 12, C, eps=eps, faults=plan, recompute=True)
    assert cnt["corrected"] == len(plan) and cnt["uncorrectable"] == 0
    assert np.array_equal(fin, clean)
    cor = ev[ev["kind"] == orc.EV_CORRECTED]
    assert {(int(e["sweep"]), int(e["z"]), int(e["y"]), int(e["x"])) for e in cor} == \
        {(int(f["sweep"]), int(f["z"]), int(f["y"]), int(f["x"])) for f in plan}
    eq10, _, _ = p.run(u0, 12, C, eps=eps, faults=plan)
    assert not np.array_equal(eq10, clean) or dtype == np.float64


def test_diagonal_pair_corrected(orc):
    """Two flips in one layer on different rows and columns: Eq.(10) cannot pair them (two
    rows, two columns: uncorrectable), evaluating the four intersections again restores the
    two corrupted points and leaves the other two as they were."""
    shape = (2, 40, 48)
    u0, C = _thermal(shape)
    p = orc.Problem(shape, orc.F32, W.THERMAL_TAPS)
    clean, _, _ = p.run(u0, 4, C, eps=1e-7)
    plan = W.make_plan([(1, 1, 8, 21, 29), (1, 1, 30, 40, 28)])
    _, _, cnt10 = p.run(u0, 4, C, eps=1e-7, faults=plan)
    assert cnt10["uncorrectable"] == 1
    fin, ev, cnt = p.run(u0, 4, C, eps=1e-7, faults=plan, recompute=True)
    assert cnt["uncorrectable"] == 0 and cnt["corrected"] == 2 and cnt["cols_flagged"] == 2
    assert np.array_equal(fin, clean)


@pytest.mark.parametrize("taps_bc", [("star2", 1), ("box", 2), ("asym", 0)])
def test_recompute_other_stencils(orc, taps_bc):
    from tests.test_oracle_memory import ASYM, BOX, STAR2
    name, bc = taps_bc
    taps = {"star2": STAR2, "box": BOX, "asym": ASYM}[name]
    shape = (5, 18, 30)
    rng = np.random.default_rng(5)
    u0 = (20 + 5 * rng.random(shape)).astype(np.float32)
    C = rng.random(shape).astype(np.float32)
    p = orc.Problem(shape, orc.F32, taps, bc=bc, bc_value=1.5)
    clean, _, _ = p.run(u0, 6, C, eps=3e-7)
    plan = W.make_plan([(1, 0, 0, 0, 29), (3, 4, 17, 29, 28), (4, 2, 5, 11, 27),
                        (4, 2, 12, 3, 29)])
    fin, ev, cnt = p.run(u0, 6, C, eps=3e-7, faults=plan, recompute=True)
    assert cnt["corrected"] == 4 and cnt["uncorrectable"] == 0
    assert np.array_equal(fin, clean)


def test_checksum_fault_unchanged_by_recompute(orc):
    """A row-only mismatch (no column flagged) is still a checksum-side fault."""
    shape = (1, 512, 4)
    u0 = np.full(shape, 100.0, np.float32) + np.random.default_rng(1).random(shape).astype(
        np.float32)
    p = orc.Problem(shape, orc.F32, W.JACOBI_TAPS)
    plan = W.make_plan([(0, 0, 100, 2, 16)])
    _, ev, cnt = p.run(u0, 1, eps=2e-5, faults=plan, recompute=True)
    assert cnt["checksum_faults"] == 1 and cnt["corrected"] == 0
