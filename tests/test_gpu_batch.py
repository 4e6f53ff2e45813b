"""Batched grids (one launch per sweep over all grids, persistent tile queue, hipGraph):
every grid of the batch against its own oracle run."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import (assert_grid_close, error_vs, event_keys, fp64_reference,
                            guarded_oracle, run_oracle, say, write_summary)

pytestmark = pytest.mark.gpu


def _run_batch(shapes, inputs, nsweeps, plan, *, eps=1e-7, graph=False, persistent=None,
               autotune=False, chunks=None, csum="f64", correction="checksum",
               taps=W.THERMAL_TAPS, mode="online", input_check=True, bc="clamp",
               bc_value=0.0):
    import torch
    from paper_1909_00709_amd import abft
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        grids = [(torch.from_numpy(u).cuda(), torch.from_numpy(c).cuda()) for u, c in inputs]
        B = abft.Batch(grids, taps, mode=mode, threshold=eps, csum=csum, stream=stream,
                       max_events=1 << 14, correction=correction, input_check=input_check,
                       bc=bc, bc_value=bc_value)
        try:
            if autotune:
                B.autotune()
            if plan is not None and len(plan):
                B.inject(plan)
            for n in (chunks or [nsweeps]):
                (B.step_graph if graph else B.step)(n)
            rep, ev = B.check()
            outs = [B.current(g)[0].cpu().numpy() for g in range(len(shapes))]
            shape = B.launch_shape()
        finally:
            B.close()
    stream.synchronize()
    return outs, ev, rep, shape


def _batch_plan(per_grid):
    rows = []
    for g, plan in per_grid.items():
        for f in plan:
            rows.append((int(f["sweep"]), int(f["z"]), int(f["y"]), int(f["x"]),
                         int(f["bit"]), 0, g))
    plan = W.empty_plan(len(rows))
    for i, r in enumerate(rows):
        for k, name in enumerate(("sweep", "z", "y", "x", "bit", "attempt", "grid")):
            plan[i][name] = r[k]
    plan.sort(order="sweep", kind="stable")
    return plan


def _check_grids(shapes, inputs, outs, ev, nsweeps, per_grid, eps, which, oracle_runs=None):
    """Each grid in `which` against its own oracle run (events exactly, values within 1e-5);
    oracle_runs[g] = (grid, events) reuses a run already made."""
    for g in which:
        u0, C = inputs[g]
        if oracle_runs is not None and g in oracle_runs:
            o, oev = oracle_runs[g]
        else:
            o, oev, _ = run_oracle(u0, W.THERMAL_TAPS, nsweeps, C=C, eps=eps,
                                   plan=per_grid.get(g))
        gev = ev[ev["grid"] == g]
        assert event_keys(gev) == event_keys(oev), g
        assert_grid_close(outs[g], o, 1e-5, f"grid {g} {shapes[g]}")


def _guarded_plans(inputs, nsweeps, per_grid, eps):
    """Per flipped grid, the oracle's run of its seeded flips with those whose relative signal
    lies in the guard band [eps/4, 4 eps] left out.  Returns (kept plans, oracle runs
    {g: (grid, events)}, records {g: fault info})."""
    kept, runs, infos = {}, {}, {}
    for g, plan in per_grid.items():
        u0, C = inputs[g]
        o, oev, _, k, info = guarded_oracle(u0, W.THERMAL_TAPS, nsweeps, plan, eps, C=C)
        runs[g] = (o, oev)
        infos[g] = info
        if len(k):
            kept[g] = k
    return kept, runs, infos


@pytest.mark.parametrize("input_check", [True, False])
@pytest.mark.parametrize("form", ["star2", "box"])
def test_batch_radius2_and_box(form, input_check):
    """Batches of radius-2 stars and of 27-point boxes: every grid against its own oracle run,
    with flips of the stored values and (with the input check) of the inputs in memory."""
    from tests.test_gpu_memory_faults import BOX, STAR2
    taps = {"star2": STAR2, "box": BOX}[form]
    shapes = W.c4_shapes(10, seed=48)
    inputs = W.c4_inputs(shapes)
    per_grid = {1: W.make_plan([(3, 0, 1, 2, 29)]),
                4: W.make_plan([(5, 1, 3, 3, 28, 0, W.FAULT_MEMORY)]),
                7: W.make_plan([(8, 2, 10, 40, 30)])}
    if not input_check:
        del per_grid[4]
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
    say("batch", form, "input_check" if input_check else "no input check")
    outs, ev, rep, _ = _run_batch(shapes, inputs, 10, plan, eps=3e-7, taps=taps,
                                  autotune=True, input_check=input_check)
    assert rep["corrected"] == 2 and rep["uncorrectable"] == 0
    assert rep["mem_corrected"] == (1 if input_check else 0)
    for g in range(len(shapes)):
        u0, C = inputs[g]
        o, oev, _ = run_oracle(u0, taps, 10, C=C, eps=3e-7, plan=per_grid.get(g),
                               input_check=input_check)
        assert event_keys(ev[ev["grid"] == g]) == event_keys(oev), g
        assert_grid_close(outs[g], o, 1e-5, f"{form} grid {g}")


def test_batch_small_mixed():
    """Twelve grids, five seeded flips (every bit the seed draws), every grid against its own
    oracle run."""
    shapes = W.c4_shapes(12, seed=44)
    inputs = W.c4_inputs(shapes)
    seeded = W.c4_plans(shapes, nsweeps=30, nflipped=5, seed=7)
    per_grid, runs, infos = _guarded_plans(inputs, 30, seeded, 1e-7)
    plan = _batch_plan(per_grid)
    say("batch small", shapes, "left out:", {g: int(i["skipped"].sum()) for g, i in infos.items()})
    outs, ev, rep, _ = _run_batch(shapes, inputs, 30, plan)
    seen = sum(int(np.sum(i["signal"][i["skipped"] == 0] > 4e-7)) for i in infos.values())
    assert rep["corrected"] == seen
    _check_grids(shapes, inputs, outs, ev, 30, per_grid, 1e-7, range(len(shapes)), runs)


def test_batch_plain_mode():
    """The unprotected batch (its own kernel variant and register budget), eager and autotuned
    in a graph, against each grid's plain oracle run; no checksum events."""
    shapes = W.c4_shapes(12, seed=46)
    inputs = W.c4_inputs(shapes)
    say("batch plain", shapes)
    a = _run_batch(shapes, inputs, 12, None, mode="none")
    b = _run_batch(shapes, inputs, 12, None, mode="none", autotune=True, graph=True,
                   chunks=[4, 8])
    assert len(a[1]) == 0 and len(b[1]) == 0
    for g in range(len(shapes)):
        u0, C = inputs[g]
        o, _, _ = run_oracle(u0, W.THERMAL_TAPS, 12, C=C, mode="none")
        assert np.array_equal(a[0][g], b[0][g]), g
        assert_grid_close(a[0][g], o, 1e-5, f"plain grid {g} {shapes[g]}")


def test_batch_dispatch_forms_and_graph_agree():
    shapes = W.c4_shapes(10, seed=45)
    inputs = W.c4_inputs(shapes)
    per_grid = {1: W.make_plan([(3, 0, 1, 2, 27)]), 7: W.make_plan([(11, 2, 5, 5, 30)])}
    plan = _batch_plan(per_grid)
    say("batch forms")
    a = _run_batch(shapes, inputs, 20, plan)
    b = _run_batch(shapes, inputs, 20, plan, autotune=True)
    c = _run_batch(shapes, inputs, 20, plan, graph=True, chunks=[5, 5, 5, 5])
    for g in range(len(shapes)):
        assert np.array_equal(a[0][g], b[0][g]) and np.array_equal(a[0][g], c[0][g]), g
    assert event_keys(a[1]) == event_keys(b[1]) == event_keys(c[1])
    assert a[2]["corrected"] == 2


@pytest.mark.parametrize("dtype,csum,input_check", [
    ("f32", "f64", False), ("f32", "f32comp", False), ("f32", "f32comp", True),
    ("f64", "f64", False), ("f64", "f64", True)])
def test_batch_dtypes_and_checksums(dtype, csum, input_check):
    """The batched variants the other batch tests leave out: the protected sweep without the
    input check (the online form the batch benchmark times), compensated-fp32 row checksums,
    and fp64 grids; autotuned and graph-captured, with mantissa and exponent flips in three
    grids, every grid against its own oracle run (events exactly; values within 1e-5 for
    fp32, 1e-12 for fp64)."""
    shapes = W.c4_shapes(10, seed=49)
    npdt = np.float32 if dtype == "f32" else np.float64
    inputs = [W.thermal_grid(nx, ny, nz, npdt, 10 + g, 110 + g)
              for g, (nz, ny, nx) in enumerate(shapes)]
    bits = (20, 26, 30) if dtype == "f32" else (44, 51, 60)
    eps, tol = (1e-7, 1e-5) if dtype == "f32" else (1e-12, 1e-12)
    per_grid = {}
    for k, g in enumerate((0, 3, 6)):
        nz, ny, nx = shapes[g]
        per_grid[g] = W.make_plan([(2 + 3 * k, (k + 1) % nz, (5 * k + 3) % ny,
                                    (11 * k + 7) % nx, bits[k])])
    plan = _batch_plan(per_grid)
    say("batch variant", dtype, csum, "input_check" if input_check else "no input check")
    outs, ev, rep, _ = _run_batch(shapes, inputs, 12, plan, eps=eps, csum=csum,
                                  input_check=input_check, autotune=True, graph=True,
                                  chunks=[6, 6])
    assert rep["corrected"] == 3 and rep["uncorrectable"] == 0, rep
    assert rep["rows_flagged"] == 3 and rep["max_noise"] < eps, rep
    for g in range(len(shapes)):
        u0, C = inputs[g]
        o, oev, _ = run_oracle(u0, W.THERMAL_TAPS, 12, C=C, eps=eps, plan=per_grid.get(g),
                               input_check=input_check)
        assert event_keys(ev[ev["grid"] == g]) == event_keys(oev), g
        assert_grid_close(outs[g], o, tol, f"{dtype} {csum} grid {g} {shapes[g]}")


@pytest.mark.parametrize("bc,input_check", [("clamp", False), ("periodic", True),
                                             ("constant", True), ("constant", False)])
def test_batch_boundary_rules_asymmetric(bc, input_check):
    """Batches under every boundary rule with asymmetric weights, so that the x-boundary terms
    of Theorem 1 do not cancel: stored-value flips in three grids and, with the input check,
    a value changed in memory in a fourth; every grid against its own oracle run."""
    from tests.test_gpu_parity import ASYM_TAPS
    shapes = W.c4_shapes(8, seed=50)
    inputs = W.c4_inputs(shapes)
    per_grid = {}
    for k, (g, bit) in enumerate(((1, 22), (4, 26), (6, 30))):
        nz, ny, nx = shapes[g]
        # row ends and an inner point, where the boundary terms and the ghosts matter
        x = (0, nx - 1, nx // 2)[k]
        per_grid[g] = W.make_plan([(1 + 3 * k, (k + 2) % nz, (7 * k + 1) % ny, x, bit)])
    if input_check:
        nz, ny, nx = shapes[2]
        per_grid[2] = W.make_plan([(4, 1, ny - 1, 3, 27, 0, W.FAULT_MEMORY)])
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
    say("batch bc", bc, "input_check" if input_check else "no input check")
    outs, ev, rep, _ = _run_batch(shapes, inputs, 10, plan, eps=3e-7, taps=ASYM_TAPS,
                                  input_check=input_check, bc=bc, bc_value=2.5, autotune=True)
    assert rep["corrected"] == 3 and rep["uncorrectable"] == 0, rep
    assert rep["mem_corrected"] == (1 if input_check else 0), rep
    for g in range(len(shapes)):
        u0, C = inputs[g]
        o, oev, _ = run_oracle(u0, ASYM_TAPS, 10, C=C, eps=3e-7, plan=per_grid.get(g), bc=bc,
                               bc_value=2.5, input_check=input_check)
        assert event_keys(ev[ev["grid"] == g]) == event_keys(oev), g
        assert_grid_close(outs[g], o, 1e-5, f"{bc} grid {g} {shapes[g]}")


def test_c4_full():
    """64 grids of 64..256 x 64..256 x 4..32 fp32, 200 sweeps, autotuned, graph-captured, one
    seeded flip in each of 8 grids (every one runs unless the oracle puts its relative signal
    in the guard band [eps/4, 4 eps]); all 64 grids against their own oracle runs, and the
    error of every grid against the fault-free fp64-storage oracle run stated (the paper's l2
    norm, Section 5.1 Eq.(11), and the largest relative error)."""
    shapes = W.c4_shapes()
    inputs = W.c4_inputs(shapes)
    seeded = W.c4_plans(shapes)
    per_grid, runs, infos = _guarded_plans(inputs, W.C4_NSWEEPS, seeded, W.C4_EPS)
    plan = _batch_plan(per_grid)
    say("C4 full", "left out:", {g: int(i["skipped"].sum()) for g, i in infos.items()})
    outs, ev, rep, shape = _run_batch(shapes, inputs, W.C4_NSWEEPS, plan, eps=W.C4_EPS,
                                      graph=True, autotune=True, chunks=[50] * 4)
    seen = {g: bool(i["signal"][0] > 4 * W.C4_EPS) for g, i in infos.items()
            if not i["skipped"][0]}
    assert rep["corrected"] == sum(seen.values())
    assert rep["rows_flagged"] == rep["corrected"]
    assert rep["max_noise"] < W.C4_EPS / 2
    for g in range(len(shapes)):
        if g not in runs:
            u0, C = inputs[g]
            o, oev, _ = run_oracle(u0, W.THERMAL_TAPS, W.C4_NSWEEPS, C=C, eps=W.C4_EPS)
            runs[g] = (o, oev)
    _check_grids(shapes, inputs, outs, ev, W.C4_NSWEEPS, per_grid, W.C4_EPS,
                 range(len(shapes)), runs)
    worst = {"l2_rel": 0.0, "max_rel": 0.0}
    worst_oracle = {"l2_rel": 0.0, "max_rel": 0.0}
    l2_sq = 0.0
    for g in range(len(shapes)):
        u0, C = inputs[g]
        ref = fp64_reference(u0, W.THERMAL_TAPS, W.C4_NSWEEPS, C=C)
        e = error_vs(outs[g], ref)
        eo = error_vs(runs[g][0], ref)
        l2_sq += e["l2_eq11"] ** 2
        for k in worst:
            worst[k] = max(worst[k], e[k])
            worst_oracle[k] = max(worst_oracle[k], eo[k])
    flips = []
    for g, i in infos.items():
        p = seeded[g][0]
        flips.append({"grid": g, "sweep": int(p["sweep"]), "bit": int(p["bit"]),
                      "signal": float(i["signal"][0]), "left_out": bool(i["skipped"][0]),
                      "corrected": bool(np.any((ev["grid"] == g) & (ev["kind"] == 2)))})
    write_summary("c4_full.json", {
        "grids": len(shapes), "sweeps": W.C4_NSWEEPS, "eps": W.C4_EPS, "flips": flips,
        "corrected": rep["corrected"], "rows_flagged": rep["rows_flagged"],
        "false_positive_rows": rep["rows_flagged"] - sum(seen.values()),
        "max_noise": rep["max_noise"], "launch_shape": shape,
        "vs_fp64_oracle": {"l2_eq11_all_grids": float(np.sqrt(l2_sq)),
                           "worst_grid_l2_rel": worst["l2_rel"],
                           "worst_grid_max_rel": worst["max_rel"]},
        "fp32_oracle_vs_fp64_oracle_worst": worst_oracle})
    # an fp32 grid after 200 sweeps stays within a few fp32 roundings per sweep of the fp64 run
    assert worst["max_rel"] < 1e-5
