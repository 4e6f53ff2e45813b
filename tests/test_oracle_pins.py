"""Pins for the CPU oracle: each check comes from outside the oracle (a library routine, exact
rational arithmetic, a closed form, a value the paper prints, or an invariant of the method).

Paper sections cited: 3.1 (Eq.(1) sweep), 3.2 (Eq.(2)-(3) checksums), 3.3 (Theorem 1,
Eq.(4)-(5)), 3.4 (Theorem 2, detection), 3.5 (Eq.(10) correction), 4 (offline), 5.1 / 5.3
(fault model, detectable bits, Table 1).
"""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.fft
import scipy.ndimage

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SCIPY_MODE = {0: "nearest", 1: "wrap", 2: "constant"}


def _kernel(taps):
    r = max([max(abs(dx), abs(dy), abs(dz)) for dx, dy, dz, _ in taps] + [0])
    K = np.zeros((2 * r + 1,) * 3)
    for dx, dy, dz, w in taps:
        K[dz + r, dy + r, dx + r] += w
    return K


def _random_taps(rng, radius, n, asym=True):
    offs = [(dx, dy, dz) for dx in range(-radius, radius + 1) for dy in range(-radius, radius + 1)
            for dz in range(-radius, radius + 1)]
    pick = rng.choice(len(offs), size=n, replace=False)
    return [(*offs[i], float(rng.uniform(-0.5, 1.0))) for i in pick]


# ----------------------------------------------------------------------------------------
# Eq.(1): the sweep equals scipy's correlate with the matching boundary mode.
# ----------------------------------------------------------------------------------------
@pytest.mark.parametrize("bc", [0, 1, 2])
@pytest.mark.parametrize("shape", [(3, 5, 7), (1, 4, 6), (2, 1, 3), (4, 6, 5)])
@pytest.mark.parametrize("radius", [1, 2])
def test_sweep_matches_scipy_correlate(orc, bc, shape, radius):
    rng = np.random.default_rng(hash((bc, shape, radius)) % 2**32)
    taps = _random_taps(rng, radius, 9)
    nz, ny, nx = shape
    if any(abs(dx) > nx or abs(dy) > ny or abs(dz) > nz for dx, dy, dz, _ in taps):
        taps = [t for t in taps if abs(t[0]) <= nx and abs(t[1]) <= ny and abs(t[2]) <= nz]
    g = 0.75
    u = rng.random(shape)
    C = rng.random(shape)
    p = orc.Problem(shape, orc.F64, taps, bc=bc, bc_value=g)
    ours = p.sweep(u, C)
    ref = scipy.ndimage.correlate(u, _kernel(taps), mode=SCIPY_MODE[bc], cval=g) + C
    np.testing.assert_allclose(ours, ref, rtol=1e-13, atol=1e-13)


def test_sweep_dyadic_exact_and_f32_rounding(orc):
    """Dyadic weights and integer data make every evaluation exact: bitwise equality.  With
    float storage the oracle rounds the exact value once."""
    rng = np.random.default_rng(7)
    taps = [(1, 0, 0, 0.125), (-1, 0, 0, 0.25), (0, 1, 0, 0.0625), (0, -1, 0, 0.5),
            (0, 0, 1, 0.03125), (0, 0, -1, 0.015625), (0, 0, 0, -0.25)]
    shape = (5, 9, 11)
    u = rng.integers(-1000, 1000, shape).astype(np.float64)
    C = rng.integers(-50, 50, shape).astype(np.float64)
    p = orc.Problem(shape, orc.F64, taps)
    ref = scipy.ndimage.correlate(u, _kernel(taps), mode="nearest") + C
    assert np.array_equal(p.sweep(u, C), ref)
    # float32 storage: one rounding of the exact value
    uf = rng.random(shape).astype(np.float32) * 300
    Cf = rng.random(shape).astype(np.float32)
    pf = orc.Problem(shape, orc.F32, W.THERMAL_TAPS)
    w32 = [(dx, dy, dz, float(np.float32(w))) for dx, dy, dz, w in W.THERMAL_TAPS]
    exact = scipy.ndimage.correlate(uf.astype(np.float64), _kernel(w32), mode="nearest") + Cf
    got = pf.sweep(uf, Cf)
    assert got.dtype == np.float32
    ulps = np.abs(got.astype(np.float64) - exact) / np.spacing(np.abs(exact).astype(np.float32))
    assert ulps.max() <= 0.5 + 1e-6


def test_paper_example_stencil_is_neighbour_average(orc):
    """Section 3.1's example set S averages the four neighbours (golden fixture)."""
    with open(os.path.join(GOLDEN, "paper_example_stencil.json")) as f:
        fx = json.load(f)
    taps = [(i, j, 0, w) for i, j, w in fx["taps_i_j_w"]]
    u = np.random.default_rng(3).random((1, 6, 6))
    out = orc.Problem((1, 6, 6), orc.F64, taps, bc=orc.BC_PERIODIC).sweep(u)
    ref = 0.25 * (np.roll(u, 1, 1) + np.roll(u, -1, 1) + np.roll(u, 1, 2) + np.roll(u, -1, 2))
    np.testing.assert_allclose(out, ref, rtol=1e-15)


# ----------------------------------------------------------------------------------------
# Eq.(2)-(3): checksums equal the exactly rounded sums (math.fsum).
# ----------------------------------------------------------------------------------------
def test_checksums_match_fsum(orc):
    rng = np.random.default_rng(11)
    shape = (3, 7, 257)
    u = rng.standard_normal(shape) * 10.0 ** rng.integers(-6, 6, shape)
    p = orc.Problem(shape, orc.F64, [])
    B = p.row_checksums(u)
    A = p.col_checksums(u)
    for z in range(shape[0]):
        for y in range(shape[1]):
            ref = math.fsum(u[z, y, :])
            assert abs(B[z, y] - ref) <= 2 * np.spacing(abs(ref)) + 1e-300
        for x in range(shape[2]):
            ref = math.fsum(u[z, :, x])
            assert abs(A[z, x] - ref) <= 2 * np.spacing(abs(ref)) + 1e-300


def test_checksums_nonfinite(orc):
    u = np.ones((1, 3, 4))
    u[0, 1, 2] = np.inf
    u[0, 2, 0] = np.nan
    p = orc.Problem(u.shape, orc.F64, [])
    B = p.row_checksums(u)
    assert B[0, 0] == 4.0 and np.isposinf(B[0, 1]) and np.isnan(B[0, 2])


# ----------------------------------------------------------------------------------------
# Theorem 1 in exact rational arithmetic: the predicted checksums equal the direct
# checksums of the next grid, for every boundary rule and asymmetric taps.
# ----------------------------------------------------------------------------------------
def _exact_next(u, C, taps, bc, g):
    nz, ny, nx = len(u), len(u[0]), len(u[0][0])

    def G(x, y, z):
        co = []
        for c, n in ((x, nx), (y, ny), (z, nz)):
            if 0 <= c < n:
                co.append(c)
            elif bc == 0:
                co.append(0 if c < 0 else n - 1)
            elif bc == 1:
                co.append(c % n)
            else:
                return g
        return u[co[2]][co[1]][co[0]]

    return [[[C[z][y][x] + sum(w * G(x + dx, y + dy, z + dz) for dx, dy, dz, w in taps)
              for x in range(nx)] for y in range(ny)] for z in range(nz)]


@pytest.mark.parametrize("seed", range(40))
def test_theorem1_exact_rational(orc, seed):
    rng = np.random.default_rng(1000 + seed)
    shape = tuple(int(v) for v in rng.integers(1, 6, 3))
    nz, ny, nx = shape
    bc = int(rng.integers(0, 3))
    radius = int(rng.integers(1, 3))
    taps = []
    for dx, dy, dz, _ in _random_taps(rng, radius, int(rng.integers(1, 8))):
        if abs(dx) <= nx and abs(dy) <= ny and abs(dz) <= nz:
            taps.append((dx, dy, dz, int(rng.integers(-8, 9)) / 8.0))
    g = int(rng.integers(-4, 5)) / 2.0
    ui = rng.integers(-64, 64, shape)
    Ci = rng.integers(-16, 16, shape)
    # exact next grid and its checksums
    uF = [[[Fraction(int(v)) for v in row] for row in lay] for lay in ui]
    CF = [[[Fraction(int(v)) for v in row] for row in lay] for lay in Ci]
    tF = [(dx, dy, dz, Fraction(w)) for dx, dy, dz, w in taps]
    nxt = _exact_next(uF, CF, tF, bc, Fraction(g))
    B_exact = np.array([[float(sum(nxt[z][y])) for y in range(ny)] for z in range(nz)])
    A_exact = np.array([[float(sum(nxt[z][y][x] for y in range(ny))) for x in range(nx)]
                        for z in range(nz)])
    p = orc.Problem(shape, orc.F64, taps, bc=bc, bc_value=g)
    u = ui.astype(np.float64)
    C = Ci.astype(np.float64)
    # dyadic data: the double evaluation is exact, so equality is exact
    assert np.array_equal(p.predict_rows_from_grid(u, C), B_exact)
    assert np.array_equal(p.predict_cols_from_grid(u, C), A_exact)
    # and the direct checksums of the oracle's own sweep agree
    nxt_o = p.sweep(u, C)
    assert np.array_equal(p.row_checksums(nxt_o), B_exact)


@pytest.mark.parametrize("seed", range(10))
def test_theorem1_general_weights(orc, seed):
    """Non-dyadic weights and real data: prediction equals the direct sums to rounding."""
    rng = np.random.default_rng(2000 + seed)
    shape = (int(rng.integers(1, 5)), int(rng.integers(2, 9)), int(rng.integers(2, 9)))
    bc = seed % 3
    taps = [t for t in _random_taps(rng, 2, 10)
            if abs(t[0]) <= shape[2] and abs(t[1]) <= shape[1] and abs(t[2]) <= shape[0]]
    u = rng.random(shape) * 100
    C = rng.random(shape)
    p = orc.Problem(shape, orc.F64, taps, bc=bc, bc_value=1.5)
    nxt = p.sweep(u, C)
    np.testing.assert_allclose(p.predict_rows_from_grid(u, C), p.row_checksums(nxt),
                               rtol=1e-12, atol=1e-10)
    np.testing.assert_allclose(p.predict_cols_from_grid(u, C), p.col_checksums(nxt),
                               rtol=1e-12, atol=1e-10)


def test_prediction_is_affine(orc):
    """Prediction minus the constant-term checksum is linear in the grid (superposition)."""
    rng = np.random.default_rng(5)
    shape = (3, 6, 9)
    taps = _random_taps(rng, 1, 7)
    p = orc.Problem(shape, orc.F64, taps, bc=orc.BC_CLAMP)
    U, V = rng.random(shape), rng.random(shape)
    a, b = 0.7, -1.3
    zero = np.zeros(shape)
    lin = lambda g: p.predict_rows_from_grid(g, zero)
    np.testing.assert_allclose(lin(a * U + b * V), a * lin(U) + b * lin(V), rtol=1e-12,
                               atol=1e-12)


# ----------------------------------------------------------------------------------------
# Closed forms for whole runs.
# ----------------------------------------------------------------------------------------
def test_jacobi_clamp_conserves_total(orc):
    u0 = W.jacobi_grid()
    p = orc.Problem(u0.shape, orc.F64, W.JACOBI_TAPS)
    fin, ev, cnt = p.run(u0, 10, mode=orc.MODE_ONLINE, eps=1e-12)
    assert cnt["rows_flagged"] == 0
    assert abs(math.fsum(fin.ravel()) / math.fsum(u0.ravel()) - 1) < 1e-14


def test_jacobi_checksum_trajectory_dct(orc):
    """Under clamp the 4-point average maps row sums by b' = b/2 + (b_{y-1} + b_{y+1})/4 with
    reflected ends, which the orthonormal DCT-II diagonalises: lambda_k = (1 + cos(pi k/n))/2."""
    u = W.jacobi_grid()
    p = orc.Problem(u.shape, orc.F64, W.JACOBI_TAPS)
    n = u.shape[1]
    lam = 0.5 + 0.5 * np.cos(np.pi * np.arange(n) / n)
    c0 = scipy.fft.dct(p.row_checksums(u)[0], type=2, norm="ortho")
    for t in range(1, 11):
        u = p.sweep(u)
        ref = scipy.fft.idct(c0 * lam ** t, type=2, norm="ortho")
        np.testing.assert_allclose(p.row_checksums(u)[0], ref, rtol=1e-13)


def test_thermal_total_heat_closed_form(orc):
    """Symmetric weights under clamp: S_{t+1} = sum(C) + q S_t with q = sum of weights."""
    nz, ny, nx = 4, 24, 32
    u0, C = W.thermal_grid(nx, ny, nz, np.float64)
    p = orc.Problem(u0.shape, orc.F64, W.THERMAL_TAPS)
    q = float(sum(Fraction(w) for *_, w in W.THERMAL_TAPS))
    sC = math.fsum(C.ravel())
    S_star = sC / (1 - q)
    S0 = math.fsum(u0.ravel())
    u = u0
    for t in range(1, 31):
        u = p.sweep(u, C)
        ref = S_star + (S0 - S_star) * q ** t
        assert abs(math.fsum(u.ravel()) / ref - 1) < 1e-13


# ----------------------------------------------------------------------------------------
# Detection (Theorem 2, Section 3.4) and the paper's detectable-bit result (Section 5.3).
# ----------------------------------------------------------------------------------------
def test_no_false_positives_fault_free(orc):
    for dtype, eps in ((orc.F32, 1e-7), (orc.F64, 1e-12)):
        u0, C = W.thermal_grid(128, 32, 4, np.float32 if dtype == orc.F32 else np.float64)
        p = orc.Problem(u0.shape, dtype, W.THERMAL_TAPS)
        _, ev, cnt = p.run(u0, 60, C, eps=eps)
        assert cnt["rows_flagged"] == 0 and len(ev) == 0
        _, ev, cnt = p.run(u0, 60, C, mode=orc.MODE_OFFLINE, period=10, eps=3 * eps)
        assert cnt["windows_flagged"] == 0 and cnt["windows_checked"] == 6


def test_paper_detectable_bits_fp32(orc):
    """Section 5.3 / Table 1: 64x64x8 fp32 tiles, 128 iterations, threshold 1e-5; flips in bits
    13..31 are detected and flips in bits 0..12 are not.  HotSpot temperatures stay in
    [256, 512), so the ambient term here holds the field near 325."""
    with open(os.path.join(GOLDEN, "paper_table1_detection.json")) as f:
        fx = json.load(f)
    t = fx["tile"]
    shape = (t["nz"], t["ny"], t["nx"])
    u0, C = W.thermal_grid(t["nx"], t["ny"], t["nz"], np.float32, t_amb=325.0)
    p = orc.Problem(shape, orc.F32, W.THERMAL_TAPS)
    rng = np.random.default_rng(99)
    rows = []
    for bit in range(fx["word_bits"]):
        for rep in range(3):
            sweep = int(rng.integers(0, fx["iterations"]))
            rows.append((sweep, int(rng.integers(0, t["nz"])), int(rng.integers(0, t["ny"])),
                         int(rng.integers(0, t["nx"])), bit))
    for r in rows:
        plan = W.make_plan([r])
        _, ev, cnt = p.run(u0, fx["iterations"], C, eps=fx["detection_threshold"], faults=plan)
        detected = cnt["rows_flagged"] > 0
        should = fx["detected_bits"]["first"] <= r[4] <= fx["detected_bits"]["last"]
        assert detected == should, (r, cnt)
        if detected:
            assert cnt["corrected"] == 1
            fl = ev[ev["kind"] == orc.EV_CORRECTED][0]
            assert (fl["sweep"], fl["z"], fl["y"], fl["x"]) == r[:4]


# ----------------------------------------------------------------------------------------
# Location and correction (Section 3.5, Eq.(10)).
# ----------------------------------------------------------------------------------------
def _integer_jacobi():
    return np.random.default_rng(0).integers(0, 1024, (1, 64, 64)).astype(np.float64)


def test_single_flip_exactly_restored(orc):
    """Integer data and the 1/4 weights keep every value and sum exact for 10 sweeps, so the
    corrected point equals the clean value bitwise and the run equals the fault-free run."""
    u0 = _integer_jacobi()
    p = orc.Problem(u0.shape, orc.F64, W.JACOBI_TAPS)
    clean, _, _ = p.run(u0, 10, eps=1e-12)
    for bit in (40, 51, 52, 57, 62):
        plan = W.make_plan([(4, 0, 17, 33, bit)])
        fin, ev, cnt = p.run(u0, 10, eps=1e-12, faults=plan)
        assert cnt["rows_flagged"] == 1 and cnt["cols_flagged"] == 1 and cnt["corrected"] == 1
        assert np.array_equal(fin, clean), bit
        none, _, _ = p.run(u0, 10, mode=orc.MODE_NONE, faults=plan)
        assert not np.array_equal(none, clean)


def test_two_flips_same_row_and_same_column(orc):
    u0 = _integer_jacobi()
    p = orc.Problem(u0.shape, orc.F64, W.JACOBI_TAPS)
    clean, _, _ = p.run(u0, 6, eps=1e-12)
    same_row = W.make_plan([(2, 0, 10, 5, 55), (2, 0, 10, 40, 53)])
    fin, ev, cnt = p.run(u0, 6, eps=1e-12, faults=same_row)
    assert cnt["corrected"] == 2 and np.array_equal(fin, clean)
    same_col = W.make_plan([(3, 0, 8, 21, 55), (3, 0, 50, 21, 60)])
    fin, ev, cnt = p.run(u0, 6, eps=1e-12, faults=same_col)
    assert cnt["corrected"] == 2 and np.array_equal(fin, clean)
    diag = W.make_plan([(3, 0, 8, 21, 55), (3, 0, 50, 30, 60)])
    fin, ev, cnt = p.run(u0, 6, eps=1e-12, faults=diag)
    assert cnt["uncorrectable"] == 1 and cnt["corrected"] == 0
    assert (ev["kind"] == orc.EV_UNCORRECTABLE).sum() == 1


def test_checksum_fault_when_columns_clean(orc):
    """Short rows, long columns: a flip seen by its row but not by its column is reported as a
    checksum-side mismatch and the grid is left alone (Figure 'fig.abft.error', scenario 2)."""
    shape = (1, 512, 4)
    u0 = np.full(shape, 100.0, np.float32) + np.random.default_rng(1).random(shape).astype(
        np.float32)
    p = orc.Problem(shape, orc.F32, W.JACOBI_TAPS)
    plan = W.make_plan([(0, 0, 100, 2, 16)])  # a 0.5 change: 1.2e-3 of a row, 1e-5 of a column
    fin, ev, cnt = p.run(u0, 1, eps=2e-5, faults=plan)
    assert cnt["rows_flagged"] == 1 and cnt["cols_flagged"] == 0
    assert cnt["checksum_faults"] == 1 and cnt["corrected"] == 0


def test_nan_flip_corrected(orc):
    """Values in [1, 2): flipping the top exponent bit gives a NaN; the mismatch test flags it
    and the partial-sum form of Eq.(10) restores a finite value."""
    shape = (2, 16, 16)
    u0 = (1.0 + np.random.default_rng(2).random(shape)).astype(np.float32)
    p = orc.Problem(shape, orc.F32, W.JACOBI_TAPS)
    clean, _, _ = p.run(u0, 3, eps=1e-6)
    plan = W.make_plan([(1, 1, 7, 9, 30)])
    fin, ev, cnt = p.run(u0, 3, eps=1e-6, faults=plan)
    assert cnt["corrected"] == 1
    corr = ev[ev["kind"] == orc.EV_CORRECTED][0]
    assert not np.isfinite(corr["a"]) and np.isfinite(corr["b"])
    np.testing.assert_allclose(fin, clean, rtol=1e-5)


def test_online_correction_error_bound_fp32(orc):
    """fp32 grid: the corrected value is within a few row-sum roundings of the clean value,
    also for exponent flips that a naive a' - (a - u) form would lose to absorption."""
    nz, ny, nx = 2, 64, 64
    u0, C = W.thermal_grid(nx, ny, nz, np.float32)
    p = orc.Problem(u0.shape, orc.F32, W.THERMAL_TAPS)
    clean, _, _ = p.run(u0, 5, C, eps=1e-7)
    for bit in (12, 20, 25, 29, 30, 31):
        plan = W.make_plan([(2, 1, 30, 40, bit)])
        fin, ev, cnt = p.run(u0, 5, C, eps=1e-7, faults=plan)
        assert cnt["corrected"] == 1, bit
        err = np.abs(fin.astype(np.float64) - clean) / np.abs(clean)
        assert err.max() < 1e-5, (bit, err.max())


# ----------------------------------------------------------------------------------------
# Offline mode (Section 4): rollback makes the run equal to the fault-free run bitwise.
# ----------------------------------------------------------------------------------------
def test_offline_rollback_bitwise(orc):
    nz, ny, nx = 4, 40, 48
    u0, C = W.thermal_grid(nx, ny, nz, np.float32)
    p = orc.Problem(u0.shape, orc.F32, W.THERMAL_TAPS)
    clean, _, _ = p.run(u0, 25, C, mode=orc.MODE_NONE)
    plan = W.make_plan([(3, 1, 5, 6, 28), (9, 2, 30, 1, 22), (22, 0, 0, 47, 31)])
    fin, ev, cnt = p.run(u0, 25, C, mode=orc.MODE_OFFLINE, period=4, eps=3e-7, faults=plan)
    assert cnt["rollbacks"] == 3 and cnt["windows_flagged"] == 3 and cnt["persistent"] == 0
    assert cnt["windows_checked"] == 7 + 3
    assert np.array_equal(fin, clean)
    rb = ev[ev["kind"] == orc.EV_ROLLBACK]
    assert sorted(rb["sweep"].tolist()) == [0, 8, 20]
    # the partial last window (sweeps 24..24) is checked too
    plan2 = W.make_plan([(24, 3, 39, 47, 30)])
    fin2, ev2, cnt2 = p.run(u0, 25, C, mode=orc.MODE_OFFLINE, period=4, eps=3e-7, faults=plan2)
    assert cnt2["rollbacks"] == 1 and np.array_equal(fin2, clean)


def test_offline_persistent_and_halt(orc):
    nz, ny, nx = 2, 16, 16
    u0, C = W.thermal_grid(nx, ny, nz, np.float64)
    p = orc.Problem(u0.shape, orc.F64, W.THERMAL_TAPS)
    plan = W.make_plan([(5, 1, 3, 3, 60, 0), (5, 1, 3, 3, 60, 1)])
    _, ev, cnt = p.run(u0, 12, C, mode=orc.MODE_OFFLINE, period=4, eps=1e-12, faults=plan)
    assert cnt["rollbacks"] == 1 and cnt["persistent"] == 1
    plan = W.make_plan([(5, 1, 3, 3, 60)])
    fin, ev, cnt = p.run(u0, 12, C, mode=orc.MODE_OFFLINE, period=4, eps=1e-12,
                         auto_correct=False, faults=plan)
    assert cnt["sweeps_done"] == 8 and cnt["rollbacks"] == 0 and cnt["windows_flagged"] == 1


def test_offline_asymmetric_weights_constant_bc(orc):
    """Boundary terms that do not cancel (asymmetric weights, constant ghosts) are carried
    through the k-fold interpolation: no false positives, and a flip is still found."""
    shape = (3, 20, 24)
    rng = np.random.default_rng(8)
    u0 = rng.random(shape) * 10
    taps = [(0, 0, 0, 0.3), (1, 0, 0, 0.25), (-1, 0, 0, 0.05), (0, 1, 0, 0.1), (0, -1, 0, 0.2),
            (0, 0, 1, 0.07), (0, 0, -1, 0.01)]
    for bc in (0, 1, 2):
        p = orc.Problem(shape, orc.F64, taps, bc=bc, bc_value=2.0)
        clean, _, cnt = p.run(u0, 20, mode=orc.MODE_OFFLINE, period=5, eps=1e-12)
        assert cnt["windows_flagged"] == 0
        plan = W.make_plan([(7, 1, 0, 23, 55)])
        fin, ev, cnt = p.run(u0, 20, mode=orc.MODE_OFFLINE, period=5, eps=1e-12, faults=plan)
        assert cnt["rollbacks"] == 1 and np.array_equal(fin, clean)


# ----------------------------------------------------------------------------------------
# Self-consistency: thread count does not change any result.
# ----------------------------------------------------------------------------------------
def test_thread_count_invariance(orc):
    nz, ny, nx = 6, 48, 40
    u0, C = W.thermal_grid(nx, ny, nz, np.float32)
    p = orc.Problem(u0.shape, orc.F32, W.THERMAL_TAPS)
    plan = W.random_plan(3, 6, 20, u0.shape, range(16, 32))
    nthr = orc.get_threads()
    try:
        orc.set_threads(1)
        a = p.run(u0, 20, C, eps=1e-7, faults=plan)
        orc.set_threads(max(2, nthr))
        b = p.run(u0, 20, C, eps=1e-7, faults=plan)
    finally:
        orc.set_threads(nthr)
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1])
    assert a[2] == b[2]


def test_validation(orc):
    assert orc.Problem((1, 4, 4), orc.F64, [(5, 0, 0, 1.0)]).validate() == -2
    assert orc.Problem((1, 4, 4), orc.F64, W.JACOBI_TAPS).validate() == 0
