"""Pins for the oracle's record of what each flip did (orc_fault_info) and for its guard band
(orc_guard), which leaves out of a parity plan the flips whose relative signal lies close to
the detection threshold (Section 3.4: the test compares a relative checksum mismatch with a
threshold; Section 5.1: the flip hits the value the sweep stores).

Each value is checked against something outside the recording code: the fault-free run's
value at the flip's site, the flipped bit pattern, exactly rounded sums (math.fsum), the
definition of the relative signal, the difference of two unprotected runs carried out in
exact (dyadic) arithmetic for the offline signal, and the run of the plan without the flip
for a flip the band leaves out.
"""
import math

import numpy as np
import pytest

import workloads as W

DYADIC_TAPS = [(0, 0, 0, 0.5), (1, 0, 0, 0.125), (-1, 0, 0, 0.125), (0, 1, 0, 0.0625),
               (0, -1, 0, 0.0625), (0, 0, 1, 0.03125), (0, 0, -1, 0.03125)]


def _flip(v, bit, dt):
    a = np.array([v], dtype=dt)
    iv = a.view(np.uint32 if dt == np.float32 else np.uint64)
    iv ^= (iv.dtype.type(1) << iv.dtype.type(bit))
    return float(a[0])


def _thermal(shape, seed=3):
    nz, ny, nx = shape
    return W.thermal_grid(nx, ny, nz, np.float32, seed, seed + 1)


@pytest.mark.parametrize("mode", ["online", "offline"])
def test_record_matches_clean_trajectory(orc, mode):
    """before = the fault-free run's value at the site after the flip's sweep, after = that
    value with the bit flipped, row and column sums = exactly rounded sums of the clean lines
    of that grid, column signal = |after - before| / |column sum|."""
    shape = (4, 24, 40)
    u0, C = _thermal(shape)
    p = orc.Problem(shape, orc.F32, W.THERMAL_TAPS)
    flips = [(2, 1, 5, 7, 27), (6, 3, 0, 39, 30), (9, 0, 23, 0, 12)]
    plan = W.make_plan(flips)
    info = np.zeros(len(plan), orc.FAULT_INFO_DTYPE)
    m = orc.MODE_ONLINE if mode == "online" else orc.MODE_OFFLINE
    p.run(u0, 12, C, mode=m, period=4, eps=1e-6, faults=plan, info=info)
    for f, (s, z, y, x, bit) in zip(info, flips):
        assert f["applied"] == 1 and f["skipped"] == 0
        clean, _, _ = p.run(u0, s + 1, C, mode=orc.MODE_NONE)
        v = float(clean[z, y, x])
        assert f["before"] == v
        assert f["after"] == _flip(v, bit, np.float32)
        assert f["row_sum"] == pytest.approx(math.fsum(clean[z, y, :].astype(float)), rel=1e-15)
        assert f["col_sum"] == pytest.approx(math.fsum(clean[z, :, x].astype(float)), rel=1e-15)
        assert f["col_signal"] == pytest.approx(abs(f["after"] - f["before"]) / abs(f["col_sum"]),
                                                rel=1e-15)
        if mode == "online":
            assert f["signal"] == pytest.approx(abs(f["after"] - f["before"]) / abs(f["row_sum"]),
                                                rel=1e-15)


def test_online_band_leaves_out_only_marginal_flips(orc):
    """Row signals below, inside and above [lo, hi]: only the flip inside is left out, and the
    run equals, bitwise with the same events, the run of the plan without it."""
    shape = (3, 16, 64)
    u0, C = _thermal(shape)
    p = orc.Problem(shape, orc.F32, W.THERMAL_TAPS)
    eps = 1e-6
    # values near 320 (ulp 2^-15), rows of 64 points: bit b gives a signal near 2^(b-29.3)
    flips = [(1, 0, 3, 9, 4), (3, 1, 8, 20, 9), (5, 2, 12, 40, 26)]
    plan = W.make_plan(flips)
    info = np.zeros(len(plan), orc.FAULT_INFO_DTYPE)
    lo, hi = eps / 4, 4 * eps
    fin, ev, cnt = p.run(u0, 8, C, eps=eps, faults=plan, guard=(lo, hi), info=info)
    sig = info["signal"]
    assert sig[0] < lo and lo <= sig[1] <= hi and sig[2] > hi, sig
    assert list(info["skipped"]) == [0, 1, 0] and list(info["applied"]) == [1, 0, 1]
    ref, rev, rcnt = p.run(u0, 8, C, eps=eps, faults=plan[[0, 2]])
    assert np.array_equal(fin, ref)
    assert np.array_equal(ev, rev) and cnt == rcnt
    # the one above the band is detected and corrected, the one below is not seen
    assert cnt["corrected"] == 1 and cnt["rows_flagged"] == 1
    # without a guard every flip is applied and the record is still written
    info2 = np.zeros(len(plan), orc.FAULT_INFO_DTYPE)
    p.run(u0, 8, C, eps=eps, faults=plan, info=info2)
    assert list(info2["applied"]) == [1, 1, 1] and not info2["skipped"].any()


def test_online_band_on_the_column_signal(orc):
    """Short rows, long columns: a flip clearly above the band for its row but inside it for
    its column is left out (the column stage would decide it marginally)."""
    shape = (1, 256, 8)
    u0, C = _thermal(shape)
    p = orc.Problem(shape, orc.F32, W.THERMAL_TAPS)
    eps = 1e-6
    info = np.zeros(1, orc.FAULT_INFO_DTYPE)
    # value ~320: bit 12 changes it by 2^(8-23+12) = 0.125; row sum ~2560, column ~82000
    plan = W.make_plan([(2, 0, 100, 3, 12)])
    p.run(u0, 4, C, eps=eps, faults=plan, guard=(eps / 4, 4 * eps), info=info)
    assert info["signal"][0] > 4 * eps and eps / 4 <= info["col_signal"][0] <= 4 * eps, info
    assert info["skipped"][0] == 1 and info["applied"][0] == 0


@pytest.mark.parametrize("bc", [0, 1, 2])
def test_offline_signal_is_the_carried_row_sum_change(orc, bc):
    """Offline, the recorded signal is the flip's change of the row sums at the window's last
    sweep.  With dyadic weights, integer data and a flip of a low mantissa bit every value is
    exact, so the change equals the difference of the row sums of two unprotected runs (with
    and without the flip) exactly; largest over the rows, over |row sum| at the flip.  Under
    the constant rule a change that reaches a row end loses part of itself through the ghost
    (the carried change leaves that out), so there the sites stay away from the x edges."""
    rng = np.random.default_rng(11 + bc)
    shape = (5, 12, 16)
    u0 = rng.integers(1, 64, shape).astype(np.float64)
    C = rng.integers(0, 4, shape).astype(np.float64)
    p = orc.Problem(shape, orc.F64, DYADIC_TAPS, bc=bc, bc_value=0.0)
    period = 6
    sites = ((0, (2, 5, 7)), (3, (0, 0, 0)), (5, (4, 11, 15)), (7, (1, 6, 3)))
    if bc == 2:
        sites = ((0, (2, 5, 7)), (3, (0, 0, 6)), (5, (4, 11, 8)), (7, (1, 6, 9)))
    for s, (z, y, x) in sites:
        # bit 45 moves a value below 64 by at least 2^-7; six sweeps of weights down to 2^-5
        # keep every value within 53 significant bits
        plan = W.make_plan([(s, z, y, x, 45)])
        info = np.zeros(1, orc.FAULT_INFO_DTYPE)
        p.run(u0, 12, C, mode=orc.MODE_OFFLINE, period=period, eps=1e-9, faults=plan,
              info=info)
        end = (s // period + 1) * period          # grid index after the window's last sweep
        faulty, _, _ = p.run(u0, end, C, mode=orc.MODE_NONE, faults=plan)
        clean, _, _ = p.run(u0, end, C, mode=orc.MODE_NONE)
        diff = p.row_checksums(faulty) - p.row_checksums(clean)
        expect = np.abs(diff).max() / abs(info["row_sum"][0])
        assert info["signal"][0] == expect, (s, info["signal"][0], expect)
        assert info["applied"][0] == 1


def test_offline_band_uses_the_carried_signal(orc):
    """A flip whose signal at its own sweep is above the band but whose carried signal at the
    window's end falls inside it is left out; the run equals the run without it."""
    shape = (4, 32, 64)
    u0, C = _thermal(shape, seed=5)
    p = orc.Problem(shape, orc.F32, W.THERMAL_TAPS)
    eps = 2e-6
    lo, hi = eps / 4, 4 * eps
    chosen = None
    for bit in range(10, 22):
        plan = W.make_plan([(0, 1, 16, 30, bit)])
        info = np.zeros(1, orc.FAULT_INFO_DTYPE)
        p.run(u0, 10, C, mode=orc.MODE_OFFLINE, period=10, eps=eps, faults=plan,
              guard=(lo, hi), info=info)
        own = abs(info["after"][0] - info["before"][0]) / abs(info["row_sum"][0])
        if own > hi and lo <= info["signal"][0] <= hi:
            chosen = (plan, info)
            break
    assert chosen is not None
    plan, info = chosen
    assert info["skipped"][0] == 1 and info["applied"][0] == 0
    fin, ev, cnt = p.run(u0, 10, C, mode=orc.MODE_OFFLINE, period=10, eps=eps, faults=plan,
                         guard=(lo, hi))
    ref, rev, rcnt = p.run(u0, 10, C, mode=orc.MODE_OFFLINE, period=10, eps=eps)
    assert np.array_equal(fin, ref) and np.array_equal(ev, rev) and cnt == rcnt


def test_non_finite_flip_has_infinite_signal(orc):
    """Exponent flips that make the value infinite or NaN are never left out."""
    shape = (2, 8, 16)
    u0, C = _thermal(shape)
    u0[1, 3, 4] = np.float32(2.0 ** 127)          # exponent field 254, mantissa 0
    u0[0, 5, 9] = np.float32(1.5 * 2.0 ** 127)    # exponent field 254, mantissa non-zero
    p = orc.Problem(shape, orc.F32, [(0, 0, 0, 1.0)])   # the identity sweep keeps the values
    plan = W.make_plan([(0, 1, 3, 4, 23), (0, 0, 5, 9, 23)])   # exponent 255: Inf, NaN
    info = np.zeros(2, orc.FAULT_INFO_DTYPE)
    p.run(u0, 1, None, eps=1e-6, faults=plan, guard=(0.0, 1e300), info=info)
    inf_i = int(np.nonzero(plan["z"] == 1)[0][0])      # make_plan orders ties by site
    assert np.isinf(info["after"][inf_i]) and np.isnan(info["after"][1 - inf_i])
    assert np.isinf(info["signal"]).all() and np.isinf(info["col_signal"]).all()
    assert list(info["skipped"]) == [0, 0] and list(info["applied"]) == [1, 1]


@pytest.mark.parametrize("mode", ["online", "offline"])
def test_piecewise_runs_equal_the_whole_run(mode):
    """The GPU tests run long oracle runs in pieces (tests/gpu_util.run_oracle with chunk):
    the pieces give the same grid, events, counters and flip records as one whole run."""
    from tests.gpu_util import run_oracle
    import oracle as O
    shape = (4, 20, 32)
    u0, C = _thermal(shape, seed=9)
    plan = W.make_plan([(1, 0, 3, 4, 28), (6, 2, 19, 31, 30), (7, 1, 0, 0, 12),
                        (13, 3, 10, 17, 26), (14, 1, 5, 5, 29, 0, W.FAULT_MEMORY),
                        (20, 0, 8, 8, 27), (20, 2, 8, 9, 3)])
    kw = dict(C=C, mode=mode, period=5, eps=1e-6, plan=plan, guard=(0.25e-6, 4e-6))
    i1 = np.zeros(len(plan), O.FAULT_INFO_DTYPE)
    i2 = np.zeros(len(plan), O.FAULT_INFO_DTYPE)
    a, aev, acnt = run_oracle(u0, W.THERMAL_TAPS, 23, info=i1, **kw)
    b, bev, bcnt = run_oracle(u0, W.THERMAL_TAPS, 23, info=i2, chunk=10, **kw)
    assert np.array_equal(a, b)
    assert np.array_equal(aev, bev) and acnt == bcnt
    assert np.array_equal(i1, i2)
    assert acnt["corrected" if mode == "online" else "rollbacks"] > 0
