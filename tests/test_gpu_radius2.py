"""Star stencils of radius 2 (13 points: the centre and two points on each side along each
axis) through the GPU path against the oracle: bitwise where every operation is exact,
every boundary rule with asymmetric weights (whose x-boundary terms of Theorem 1 do not
cancel), online location and correction, offline rollback, the autotuned and graph-captured
forms, and the 1024 x 1024 x 128 fp32 grid at full size.  Bars as for radius 1: fp64 grids
within 1e-12, fp32 grids within 1e-5, detection and location events equal."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import assert_grid_close, event_keys, run_gpu, run_oracle, say

pytestmark = pytest.mark.gpu


def star2(c, x1, x2, y1, y2, z1, z2, asym=1.0):
    """Radius-2 star taps (dx, dy, dz, w); asym scales the plus side of every axis."""
    taps = [(0, 0, 0, c)]
    for d, (w1, w2) in enumerate(((x1, x2), (y1, y2), (z1, z2))):
        for dist, w in ((1, w1), (2, w2)):
            for sg in (-1, 1):
                off = [0, 0, 0]
                off[d] = sg * dist
                taps.append((off[0], off[1], off[2], w * (asym if sg > 0 else 1.0)))
    return tuple(taps)


DYADIC2 = star2(0.5, 0.0625, 0.03125, 0.0625, 0.03125, 0.0625, 0.03125)
# fourth-order diffusion, u + 0.05 * (the 5-point second difference along each axis) / 12
DIFF4 = star2(1 - 3 * 0.05 * 30 / 12, 0.05 * 16 / 12, -0.05 / 12, 0.05 * 16 / 12, -0.05 / 12,
              0.05 * 16 / 12, -0.05 / 12)
ASYM2 = star2(0.3, 0.12, 0.03, 0.1, 0.02, 0.06, 0.01, asym=1.5)


@pytest.mark.parametrize("dtype,nsweeps", [(np.float64, 5), (np.float32, 3)])
@pytest.mark.parametrize("shape", [(6, 37, 64), (3, 20, 1024), (4, 9, 7), (5, 16, 130)])
@pytest.mark.parametrize("bc", ["clamp", "periodic"])
def test_radius2_dyadic_bitwise(dtype, nsweeps, shape, bc):
    if dtype == np.float32 and shape[2] == 130:
        shape = (5, 16, 132)
    rng = np.random.default_rng(23)
    u0 = rng.integers(0, 64, shape).astype(dtype)
    C = rng.integers(-4, 4, shape).astype(dtype)
    eps = 1e-12 if dtype == np.float64 else 1e-7
    say("radius 2 dyadic", dtype.__name__, shape, bc)
    g, gev, grep, _ = run_gpu(u0, DYADIC2, nsweeps, C=C, eps=eps, bc=bc)
    o, oev, ocnt = run_oracle(u0, DYADIC2, nsweeps, C=C, eps=eps, bc=bc)
    assert grep["rows_flagged"] == 0 and ocnt["rows_flagged"] == 0
    assert np.array_equal(g, o)


CASES = [
    ((5, 13, 9), np.float64, "clamp"),
    ((4, 17, 100), np.float32, "periodic"),
    ((3, 33, 252), np.float32, "constant"),
    ((6, 19, 260), np.float64, "constant"),
    ((2, 40, 96), np.float64, "periodic"),
    ((7, 70, 520), np.float32, "clamp"),
    ((9, 11, 301), np.float32, "periodic"),
]


@pytest.mark.parametrize("shape,dtype,bc", CASES)
def test_radius2_online_boundaries(shape, dtype, bc):
    nz, ny, nx = shape
    rng = np.random.default_rng(nx * 7 + ny)
    u0 = (50 + 10 * rng.random(shape)).astype(dtype)
    C = rng.random(shape).astype(dtype)
    f64 = dtype == np.float64
    eps = 1e-12 if f64 else 1e-7 * max(1.0, (512.0 / min(nx, ny)) ** 0.5)
    bit = 60 if f64 else 28
    plan = W.make_plan([(3, nz // 2, ny - 1, nx - 1, bit), (6, 0, 1, 0, bit - 3)])
    say("radius 2 online", shape, dtype.__name__, bc)
    g, gev, grep, _ = run_gpu(u0, ASYM2, 9, C=C, eps=eps, bc=bc, bc_value=2.5, plan=plan)
    o, oev, ocnt = run_oracle(u0, ASYM2, 9, C=C, eps=eps, bc=bc, bc_value=2.5, plan=plan)
    assert event_keys(gev) == event_keys(oev)
    assert grep["corrected"] == 2
    assert_grid_close(g, o, 1e-12 if f64 else 1e-5, f"radius 2 {shape} {bc}")


@pytest.mark.parametrize("bc", ["clamp", "constant", "periodic"])
def test_radius2_offline(bc):
    """Windows of 5 with asymmetric taps: the per-sweep x-boundary terms enter the 5-fold
    interpolation; two flips roll two windows back, and the run equals the fault-free one."""
    shape = (6, 40, 96)
    rng = np.random.default_rng(8)
    u0 = 10 * rng.random(shape)
    plan = W.make_plan([(7, 1, 0, 95, 55), (13, 3, 39, 0, 62)])
    say("radius 2 offline", bc)
    g, gev, grep, _ = run_gpu(u0, ASYM2, 23, mode="offline", period=5, eps=1e-12, bc=bc,
                              bc_value=2.0, plan=plan)
    o, oev, ocnt = run_oracle(u0, ASYM2, 23, mode="offline", period=5, eps=1e-12, bc=bc,
                              bc_value=2.0, plan=plan)
    assert event_keys(gev) == event_keys(oev)
    assert grep["rollbacks"] == 2 and grep["windows_checked"] == ocnt["windows_checked"]
    assert np.array_equal(g, run_gpu(u0, ASYM2, 23, mode="none", bc=bc, bc_value=2.0)[0])
    assert_grid_close(g, o, 1e-12, "radius 2 offline")


def test_radius2_offline_long_window():
    """A 20-sweep window: the interpolation runs in chunks (8 steps each at radius 2)."""
    shape = (8, 48, 128)
    u0, C = W.thermal_grid(128, 48, 8, np.float64)
    plan = W.make_plan([(25, 4, 20, 64, 58)])
    say("radius 2 offline, period 20")
    g, gev, grep, _ = run_gpu(u0, DIFF4, 41, C=C, mode="offline", period=20, eps=1e-12,
                              plan=plan)
    o, oev, ocnt = run_oracle(u0, DIFF4, 41, C=C, mode="offline", period=20, eps=1e-12,
                              plan=plan)
    assert event_keys(gev) == event_keys(oev)
    assert grep["rollbacks"] == 1
    assert_grid_close(g, o, 1e-12, "radius 2 period 20")


def test_radius2_fp32_thermal_autotuned_graph():
    nz, ny, nx = 16, 96, 512
    u0, C = W.thermal_grid(nx, ny, nz, np.float32)
    plan = W.random_plan(78, 8, 40, (nz, ny, nx), list(range(16, 31)))
    say("radius 2 fp32, autotuned, graph")
    g, gev, grep, shape = run_gpu(u0, DIFF4, 40, C=C, eps=2e-7, plan=plan, autotune=True,
                                  graph=True, chunks=[10] * 4)
    o, oev, ocnt = run_oracle(u0, DIFF4, 40, C=C, eps=2e-7, plan=plan)
    assert event_keys(gev) == event_keys(oev)
    assert grep["corrected"] == ocnt["corrected"] == len(plan)
    assert_grid_close(g, o, 1e-5, "radius 2 fp32 thermal")


def test_radius2_fullsize_parity():
    """The 1024 x 1024 x 128 fp32 grid, 10 sweeps online with two flips, autotuned."""
    u0, C = W.C5.inputs()
    plan = W.make_plan([(2, 64, 512, 1023, 30), (7, 127, 0, 0, 27)])
    say("radius 2 full size")
    g, gev, grep, _ = run_gpu(u0, DIFF4, 10, C=C, eps=2e-7, plan=plan, autotune=True)
    o, oev, ocnt = run_oracle(u0, DIFF4, 10, C=C, eps=2e-7, plan=plan)
    assert event_keys(gev) == event_keys(oev)
    assert grep["corrected"] == 2
    assert_grid_close(g, o, 1e-5, "radius 2 full size")


def test_radius2_rejected_where_unsupported():
    import torch
    from paper_1909_00709_amd import abft
    with pytest.raises(abft.AbftError):  # distance-2 x taps on rows of length 1
        abft.Stencil(torch.zeros((2, 8, 1), device="cuda", dtype=torch.float64), DYADIC2)
    u = torch.zeros((2, 8, 1), device="cuda")
    with pytest.raises(abft.AbftError):  # the same in a batch
        abft.Batch([(u, None)], DYADIC2)


@pytest.mark.parametrize("form", ["star2", "box"])
@pytest.mark.parametrize("mode,input_check", [("online", False), ("online", True),
                                              ("offline", False)])
def test_f32comp_radius2_and_box(form, mode, input_check):
    """Compensated-fp32 row checksums with the radius-2 star and the 27-point box (kernel
    variants of their own): an fp32 thermal grid with asymmetric weights, flips at a row's
    first and last points and inside, online location and correction (with and without the
    input check) or offline rollback, against the oracle (fp64 checksums; events equal, every
    flip far above the threshold; values within 1e-5)."""
    from tests.test_gpu_memory_faults import BOX, STAR2
    taps = {"star2": STAR2, "box": BOX}[form]
    u0, C = W.thermal_grid(260, 33, 6, np.float32, 3, 4)
    plan = W.make_plan([(1, 2, 0, 0, 26), (4, 4, 17, 259, 22), (7, 1, 32, 130, 30)])
    eps = 3e-7 if mode == "online" else 2e-6
    kw = dict(C=C, eps=eps, plan=plan, mode=mode, period=3, input_check=input_check)
    say("f32comp", form, mode, input_check)
    g, gev, grep, _ = run_gpu(u0, taps, 9, csum="f32comp", autotune=True, **kw)
    o, oev, ocnt = run_oracle(u0, taps, 9, **kw)
    if mode == "online":
        assert grep["corrected"] == 3 and ocnt["corrected"] == 3, (grep, ocnt)
    else:
        assert grep["rollbacks"] == 3 and ocnt["rollbacks"] == 3, (grep, ocnt)
    assert grep["uncorrectable"] == 0 and grep["persistent"] == 0
    assert event_keys(gev) == event_keys(oev)
    assert_grid_close(g, o, 1e-5, f"f32comp {form} {mode}")


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("mode,input_check", [("online", False), ("online", True),
                                              ("offline", False), ("none", False)])
def test_radius2_wide_blocks_forced(mode, input_check, dtype, tmp_path):
    """Radius-2 sweeps in blocks of 8 wavefronts (8 rows of 1024 fp32 or 512 fp64 points, 64
    lanes of four 16-byte chunks per row), forced through the tuning cache for every variant
    (the autotuner may prefer 4-wavefront blocks for some): online location and correction
    with and without the input check, offline rollback (the one-launch recompute in the same
    block shape), and plain sweeps, against the oracle; a ragged last row block and a ragged
    last slab."""
    f32 = dtype == "f32"
    nx = 1024 if f32 else 512
    u0, C = W.thermal_grid(nx, 21, 7, np.float32 if f32 else np.float64, 5, 6)
    mcode = {"none": 0, "online": 1, "offline": 2}[mode]
    tags = "r2 ic" if input_check else "r2"
    cache = tmp_path / "wide.tune"
    cache.write_text(f"{0 if f32 else 1} {nx} 21 7 {mcode} 0 {tags} 64 4 {4 if f32 else 2} 4 1 8\n")
    bits = (26, 22, 30) if f32 else (60, 51, 44)
    plan = W.make_plan([(1, 2, 0, 0, bits[0]), (4, 6, 20, nx - 1, bits[1]),
                        (7, 1, 9, 317, bits[2])])
    if f32:
        eps, tol = (3e-7 if mode != "offline" else 2e-6), 1e-5
    else:
        eps, tol = 1e-12, 1e-12
    kw = dict(C=C, eps=eps, mode=mode, period=3, input_check=input_check)
    if mode != "none":
        kw["plan"] = plan
    say("radius 2 wide blocks", mode, input_check)
    g, gev, grep, shape = run_gpu(u0, ASYM2, 9, tuning_cache=str(cache), **kw)
    assert shape[0] == 8, shape  # 8 rows per block: the cached 8-wavefront shape is in use
    o, oev, ocnt = run_oracle(u0, ASYM2, 9, **kw)
    if mode == "online":
        assert grep["corrected"] == 3 and ocnt["corrected"] == 3, (grep, ocnt)
    elif mode == "offline":
        assert grep["rollbacks"] == 3 and ocnt["rollbacks"] == 3, (grep, ocnt)
    assert event_keys(gev) == event_keys(oev)
    assert_grid_close(g, o, tol, f"radius 2 wide blocks {dtype} {mode}")


@pytest.mark.parametrize("shape,drop_axis", [((1, 48, 96), 2), ((6, 1, 64), 1)])
@pytest.mark.parametrize("bc", ["periodic", "clamp", "constant"])
def test_radius2_axis_of_length_one(shape, drop_axis, bc):
    """A radius-2 star on a grid with an axis of length 1 that carries no distance-2 tap (a 2D
    grid, or a single row per layer): the plane and halo-row coordinates two steps outside
    that axis map back onto it under every boundary rule.  Online, with flips, against the
    oracle."""
    taps = tuple(t for t in ASYM2 if abs((t[0], t[1], t[2])[drop_axis]) < 2)
    nz, ny, nx = shape
    rng = np.random.default_rng(nz * 100 + ny)
    u0 = 50 + 10 * rng.random(shape)
    C = rng.random(shape)
    plan = W.make_plan([(2, nz - 1, ny - 1, nx - 1, 60), (5, 0, 0, 1, 57)])
    say("radius 2 axis of length 1", shape, bc)
    g, gev, grep, _ = run_gpu(u0, taps, 8, C=C, eps=1e-12, bc=bc, bc_value=2.5, plan=plan)
    o, oev, ocnt = run_oracle(u0, taps, 8, C=C, eps=1e-12, bc=bc, bc_value=2.5, plan=plan)
    assert event_keys(gev) == event_keys(oev)
    assert grep["corrected"] == ocnt["corrected"] == 2
    assert_grid_close(g, o, 1e-12, f"radius 2 {shape} {bc}")
