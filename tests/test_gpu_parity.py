"""GPU parity: the HIP path through the C-ABI against the CPU oracle on the same seeded inputs.

Bars (stated in the workloads' description): fp64 grids within 1e-12 relative, fp32 grids
within 1e-5 relative (both the l2 ratio and the max-abs ratio); detection and location events
equal exactly.  Flips whose relative signal falls within [eps/4, 4 eps] are kept out of the
fault plans (guard band): there both sides are right to decide either way under rounding.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import (assert_grid_close, corrected_values, event_keys, guarded_oracle,
                            run_gpu, run_oracle, say)

pytestmark = pytest.mark.gpu

DYADIC_TAPS = ((0, 0, 0, 0.5), (-1, 0, 0, 0.125), (1, 0, 0, 0.125), (0, -1, 0, 0.0625),
               (0, 1, 0, 0.0625), (0, 0, -1, 0.0625), (0, 0, 1, 0.0625))
ASYM_TAPS = ((0, 0, 0, 0.3), (1, 0, 0, 0.25), (-1, 0, 0, 0.05), (0, 1, 0, 0.1),
             (0, -1, 0, 0.2), (0, 0, 1, 0.07), (0, 0, -1, 0.01))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    from paper_1909_00709_amd import abft  # noqa: F401  (fails loudly without the library)


# ---------------------------------------------------------------------------------------
# C1: 2D Jacobi 64x64 fp64, 10 sweeps, one flip at bit 40..62, detected and corrected.
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("bit", range(40, 63))
def test_c1_jacobi_flip(bit):
    u0, C = W.C1.inputs()
    plan = W.c1_plan(bit)
    say("C1", "bit", bit, plan.tolist())
    g, gev, grep, _ = run_gpu(u0, W.JACOBI_TAPS, W.C1.nsweeps, eps=W.C1.eps, plan=plan)
    o, oev, ocnt = run_oracle(u0, W.JACOBI_TAPS, W.C1.nsweeps, eps=W.C1.eps, plan=plan)
    assert event_keys(gev) == event_keys(oev)
    assert grep["corrected"] == ocnt["corrected"] == 1
    assert_grid_close(g, o, 1e-12, f"C1 bit {bit}")
    gc, oc = corrected_values(gev), corrected_values(oev)
    for k in oc:
        assert abs(gc[k] - oc[k]) <= 1e-12 * abs(oc[k]) + 1e-15


# ---------------------------------------------------------------------------------------
# Bitwise agreement where every operation is exact (dyadic weights, integer data).
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("dtype,nsweeps", [(np.float64, 8), (np.float32, 3)])
@pytest.mark.parametrize("shape", [(5, 37, 64), (3, 20, 1024), (2, 9, 7)])
def test_dyadic_bitwise(dtype, nsweeps, shape):
    rng = np.random.default_rng(17)
    u0 = rng.integers(0, 1000, shape).astype(dtype)
    C = rng.integers(-8, 8, shape).astype(dtype)
    eps = 1e-12 if dtype == np.float64 else 1e-7
    say("dyadic", dtype.__name__, shape)
    g, gev, grep, _ = run_gpu(u0, DYADIC_TAPS, nsweeps, C=C, eps=eps)
    o, oev, ocnt = run_oracle(u0, DYADIC_TAPS, nsweeps, C=C, eps=eps)
    assert grep["rows_flagged"] == 0 and ocnt["rows_flagged"] == 0
    assert np.array_equal(g, o)


# ---------------------------------------------------------------------------------------
# Ragged shapes, every boundary rule, asymmetric weights, both dtypes, one flip.
# ---------------------------------------------------------------------------------------
CASES = [
    # shape (nz, ny, nx), dtype, bc
    ((5, 13, 7), np.float64, "clamp"),
    ((4, 17, 100), np.float32, "periodic"),
    ((3, 33, 252), np.float32, "constant"),
    ((6, 19, 260), np.float64, "clamp"),
    ((1, 40, 96), np.float64, "periodic"),
    ((7, 70, 520), np.float32, "clamp"),
    ((2, 5, 1024), np.float32, "constant"),
    ((9, 11, 300), np.float32, "periodic"),
]


@pytest.mark.parametrize("shape,dtype,bc", CASES)
def test_ragged_shapes_and_boundaries(shape, dtype, bc):
    nz, ny, nx = shape
    rng = np.random.default_rng(nx * 31 + ny)
    u0 = (50 + 10 * rng.random(shape)).astype(dtype)
    C = rng.random(shape).astype(dtype)
    f64 = dtype == np.float64
    # fp32 rounding of a point is a few ulps (fma chain); a line of n points averages it only
    # by sqrt(n), so the threshold grows for the short extents of these cases (Section 3.4:
    # the threshold depends on the size of the checked block)
    eps = 1e-12 if f64 else 1e-7 * max(1.0, (512.0 / min(nx, ny)) ** 0.5)
    bit = 60 if f64 else 28
    plan = W.make_plan([(3, nz // 2, ny - 1, nx - 1, bit), (6, 0, 0, 0, bit - 3)])
    say("ragged", shape, dtype.__name__, bc)
    g, gev, grep, _ = run_gpu(u0, ASYM_TAPS, 9, C=C, eps=eps, bc=bc, bc_value=2.5, plan=plan)
    o, oev, ocnt = run_oracle(u0, ASYM_TAPS, 9, C=C, eps=eps, bc=bc, bc_value=2.5, plan=plan)
    assert event_keys(gev) == event_keys(oev)
    assert grep["corrected"] == 2
    assert_grid_close(g, o, 1e-12 if f64 else 1e-5, f"{shape} {bc}")


# ---------------------------------------------------------------------------------------
# fp32 thermal grids, both checksum accumulations, several flips.
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("csum", ["f64", "f32comp"])
def test_fp32_thermal_online(csum):
    nz, ny, nx = 16, 96, 512
    u0, C = W.thermal_grid(nx, ny, nz, np.float32)
    plan = W.random_plan(77, 12, 40, (nz, ny, nx), list(range(14, 32)))
    say("fp32 thermal", csum)
    g, gev, grep, _ = run_gpu(u0, W.THERMAL_TAPS, 40, C=C, eps=1e-7, csum=csum, plan=plan)
    o, oev, ocnt = run_oracle(u0, W.THERMAL_TAPS, 40, C=C, eps=1e-7, plan=plan)
    assert event_keys(gev) == event_keys(oev)
    assert grep["corrected"] == ocnt["corrected"] == len(plan)
    assert grep["max_noise"] < 1e-7 / 4
    assert_grid_close(g, o, 1e-5, f"thermal {csum}")


# ---------------------------------------------------------------------------------------
# C2: 3D thermal 512x512x8 fp64, 100 sweeps, online and offline (k = 10), 0..10 flips.
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("mode", ["online", "offline"])
@pytest.mark.parametrize("nflips", [0, 1, 5, 10])
def test_c2(mode, nflips):
    """Every seeded flip runs unless the oracle's own run puts its relative signal inside the
    guard band [eps/4, 4 eps] (there both sides may decide either way under rounding)."""
    u0, C = W.C2.inputs()
    eps = W.C2.eps
    full = W.c2_plan(nflips)
    o, oev, ocnt, plan, info = guarded_oracle(u0, W.THERMAL_TAPS, W.C2.nsweeps, full, eps, C=C,
                                              mode=mode, period=10)
    say("C2", mode, nflips, plan.tolist(), "left out:", int(info["skipped"].sum()))
    g, gev, grep, _ = run_gpu(u0, W.THERMAL_TAPS, W.C2.nsweeps, C=C, eps=eps, mode=mode,
                              period=10, plan=plan)
    assert event_keys(gev) == event_keys(oev)
    for k in ("rows_flagged", "corrected", "windows_flagged", "rollbacks", "persistent"):
        assert grep[k] == ocnt[k], k
    assert_grid_close(g, o, 1e-12, f"C2 {mode} {nflips}")
    kept = info[info["skipped"] == 0]
    if mode == "offline" and np.all(kept["signal"] > 4 * eps):
        # every flip was seen, so the rollbacks erase all of them bitwise
        clean, _, _, _ = run_gpu(u0, W.THERMAL_TAPS, W.C2.nsweeps, C=C, mode="none")
        assert np.array_equal(g, clean)


# ---------------------------------------------------------------------------------------
# Offline details: boundary terms that do not cancel, partial windows, manual correction.
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("bc", ["clamp", "constant", "periodic"])
def test_offline_asymmetric(bc):
    shape = (4, 40, 96)
    rng = np.random.default_rng(5)
    u0 = (10 * rng.random(shape))
    plan = W.make_plan([(7, 1, 0, 95, 55), (13, 3, 39, 0, 62)])
    say("offline asym", bc)
    g, gev, grep, _ = run_gpu(u0, ASYM_TAPS, 23, mode="offline", period=5, eps=1e-12, bc=bc,
                              bc_value=2.0, plan=plan)
    o, oev, ocnt = run_oracle(u0, ASYM_TAPS, 23, mode="offline", period=5, eps=1e-12, bc=bc,
                              bc_value=2.0, plan=plan)
    assert event_keys(gev) == event_keys(oev)
    assert grep["rollbacks"] == 2 and grep["windows_checked"] == ocnt["windows_checked"]
    assert np.array_equal(g, run_gpu(u0, ASYM_TAPS, 23, mode="none", bc=bc, bc_value=2.0)[0])
    assert_grid_close(g, o, 1e-12, "offline asym")


def test_offline_manual_correct():
    import torch
    from paper_1909_00709_amd import abft
    nz, ny, nx = 4, 64, 128
    u0, C = W.thermal_grid(nx, ny, nz, np.float64)
    plan = W.make_plan([(12, 2, 10, 20, 58)])
    say("offline manual")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        S = abft.Stencil(torch.from_numpy(u0).cuda(), W.THERMAL_TAPS, C=torch.from_numpy(C).cuda(),
                         mode="offline", period=5, threshold=1e-12, auto_correct=False,
                         stream=stream)
        S.inject(plan)
        S.step(30)
        rep, ev = S.check()
        assert rep["pending"] > 0 and rep["sweeps_done"] == 15 and rep["sweeps_skipped"] == 15
        with pytest.raises(abft.AbftError):
            S.step(1)
        s, rep, ev = S.correct()
        assert s == abft.ABFT_OK and rep["rollbacks"] == 1 and rep["pending"] == 0
        S.step(rep["sweeps_skipped"])
        rep, ev = S.check()
        g = S.current()[0].cpu().numpy()
        S.close()
    o, oev, ocnt = run_oracle(u0, W.THERMAL_TAPS, 30, C=C, mode="offline", period=5, eps=1e-12,
                              plan=plan)
    assert_grid_close(g, o, 1e-12, "offline manual")


def test_online_manual_correct():
    import torch
    from paper_1909_00709_amd import abft
    nz, ny, nx = 3, 48, 256
    u0, C = W.thermal_grid(nx, ny, nz, np.float32)
    plan = W.make_plan([(4, 1, 7, 100, 27)])
    say("online manual")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        S = abft.Stencil(torch.from_numpy(u0).cuda(), W.THERMAL_TAPS, C=torch.from_numpy(C).cuda(),
                         threshold=1e-7, auto_correct=False, stream=stream)
        S.inject(plan)
        S.step(5)
        rep, ev = S.check()
        assert rep["pending"] == 1 and rep["rows_flagged"] == 1 and rep["corrected"] == 0
        s, rep, ev = S.correct()
        assert s == abft.ABFT_OK and rep["corrected"] == 1 and rep["pending"] == 0
        S.step(5)
        g = S.current()[0].cpu().numpy()
        S.close()
    o, _, _ = run_oracle(u0, W.THERMAL_TAPS, 10, C=C, eps=1e-7, plan=plan)
    assert_grid_close(g, o, 1e-5, "online manual")


def test_uncorrectable_and_checksum_fault():
    nz, ny, nx = 2, 64, 64
    u0 = np.random.default_rng(0).integers(0, 1024, (nz, ny, nx)).astype(np.float64)
    plan = W.make_plan([(2, 1, 8, 21, 55), (2, 1, 50, 30, 60), (4, 0, 5, 5, 57),
                        (4, 0, 5, 40, 52)])
    say("uncorrectable")
    g, gev, grep, _ = run_gpu(u0, W.JACOBI_TAPS, 6, eps=1e-12, plan=plan)
    o, oev, ocnt = run_oracle(u0, W.JACOBI_TAPS, 6, eps=1e-12, plan=plan)
    assert grep["uncorrectable"] == ocnt["uncorrectable"] == 1
    assert grep["corrected"] == ocnt["corrected"] == 2
    assert event_keys(gev) == event_keys(oev)
    assert_grid_close(g, o, 1e-12, "uncorrectable")
    # short rows, long columns: a row-only mismatch is a checksum-side fault
    shape = (1, 512, 4)
    u1 = (100.0 + np.random.default_rng(1).random(shape)).astype(np.float32)
    plan = W.make_plan([(0, 0, 100, 2, 16)])
    g, gev, grep, _ = run_gpu(u1, W.JACOBI_TAPS, 1, eps=2e-5, plan=plan)
    assert grep["checksum_faults"] == 1 and grep["corrected"] == 0


# ---------------------------------------------------------------------------------------
# Graph replays and determinism.
# ---------------------------------------------------------------------------------------
def test_graph_replay_matches_eager():
    import torch
    from paper_1909_00709_amd import abft
    nz, ny, nx = 8, 128, 512
    u0, C = W.thermal_grid(nx, ny, nz, np.float32)
    plan = W.make_plan([(3, 2, 5, 7, 29), (17, 6, 100, 400, 25), (33, 0, 0, 511, 31)])
    say("graph replay")
    eager, eev, erep, _ = run_gpu(u0, W.THERMAL_TAPS, 40, C=C, eps=1e-7, plan=plan)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        S = abft.Stencil(torch.from_numpy(u0).cuda(), W.THERMAL_TAPS, C=torch.from_numpy(C).cuda(),
                         threshold=1e-7, stream=stream)
        S.inject(plan)
        grids = []
        for rep in range(4):  # the same 10-sweep graph replayed, eager work in between
            S.step_graph(10)
            cur, t = S.current()
            grids.append(cur.cpu().numpy())
            _ = (cur * 2).sum().item()
        rep, ev = S.check()
        S.close()
    assert rep["corrected"] == 3
    assert np.array_equal(grids[-1], eager)
    assert event_keys(ev) == event_keys(eev)
    for i, n in enumerate((10, 20, 30)):
        ref, _, _, _ = run_gpu(u0, W.THERMAL_TAPS, n, C=C, eps=1e-7, plan=plan)
        assert np.array_equal(grids[i], ref)


def test_deterministic_repeat():
    u0, C = W.thermal_grid(512, 256, 16, np.float32)
    plan = W.random_plan(9, 5, 20, (16, 256, 512), list(range(20, 32)))
    a = run_gpu(u0, W.THERMAL_TAPS, 20, C=C, eps=1e-7, plan=plan, csum="f32comp")
    b = run_gpu(u0, W.THERMAL_TAPS, 20, C=C, eps=1e-7, plan=plan, csum="f32comp")
    assert np.array_equal(a[0], b[0])
    assert event_keys(a[1]) == event_keys(b[1])
    assert corrected_values(a[1]) == corrected_values(b[1])


def test_offline_fp32_compensated():
    """fp32 grid, offline windows with compensated-fp32 direct checksums."""
    nz, ny, nx = 16, 128, 1024
    u0, C = W.thermal_grid(nx, ny, nz, np.float32)
    plan = W.make_plan([(4, 3, 17, 900, 29), (26, 9, 127, 0, 27)])
    say("offline fp32 f32comp")
    g, gev, grep, _ = run_gpu(u0, W.THERMAL_TAPS, 30, C=C, mode="offline", period=10,
                              eps=W.C5.eps, csum="f32comp", plan=plan)
    o, oev, ocnt = run_oracle(u0, W.THERMAL_TAPS, 30, C=C, mode="offline", period=10,
                              eps=W.C5.eps, plan=plan)
    assert event_keys(gev) == event_keys(oev)
    assert grep["rollbacks"] == 2 and grep["max_noise"] < W.C5.eps / 4
    clean = run_gpu(u0, W.THERMAL_TAPS, 30, C=C, mode="none")[0]
    assert np.array_equal(g, clean)
    assert_grid_close(g, o, 1e-5, "offline fp32")
