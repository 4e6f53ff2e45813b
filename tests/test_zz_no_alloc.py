"""The allocation-free entry point (abft_stencil_run_noalloc) through the C ABI against the
existing entry points it stands for (abft_stencil_init, _inject, _step, _check): the same
kernels and the same default launch shape, so the grid, the events and the report must be
bitwise equal; two calls in a row, the second on a smaller grid (the static workspace keeps
the first call's contents), and each result also against the oracle."""
import ctypes

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import assert_grid_close, event_keys, run_oracle, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def abft():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    from paper_1909_00709_amd import abft as A
    return A


def _report(abft, cap):
    ev = (abft.AbftEvent * cap)()
    rep = abft.AbftReport()
    rep.events = ctypes.cast(ev, ctypes.POINTER(abft.AbftEvent))
    rep.events_cap = cap
    return rep, ev


def _as_dict(abft, rep, ev):
    out = {f: getattr(rep, f) for f in abft.REPORT_COUNTERS}
    out["max_noise"] = rep.max_noise
    arr = np.frombuffer(ev, dtype=abft.EVENT_DTYPE, count=len(ev))[:rep.nevents].copy()
    return out, arr


def _existing(abft, u0, C, plan, nsweeps, mode, input_check, stream):
    """init + inject + step + check + destroy."""
    import torch
    with torch.cuda.stream(stream):
        S = abft.Stencil(torch.from_numpy(u0).cuda(), W.THERMAL_TAPS,
                         C=torch.from_numpy(C).cuda(), mode=mode, threshold=1e-7,
                         input_check=input_check, max_events=1024, stream=stream)
        try:
            if plan is not None:
                S.inject(plan)
            S.step(nsweeps)
            rep, ev = S.check()
            g = S.current()[0].cpu().numpy()
        finally:
            S.close()
    return g, rep, ev


def _noalloc(abft, u0, C, plan, nsweeps, mode, input_check, stream):
    import torch
    with torch.cuda.stream(stream):
        ut = torch.from_numpy(u0).cuda()
        u1 = torch.empty_like(ut)
        Ct = torch.from_numpy(C).cuda()
        prob = abft.make_problem(u0.shape, abft.ABFT_F32, W.THERMAL_TAPS, ut.data_ptr(),
                                 u1.data_ptr(), None, Ct.data_ptr())
        opts = abft.make_options(mode, threshold=1e-7, max_events=1024,
                                 input_check=input_check)
        rep, ev = _report(abft, 1024)
        s = abft.abft_stencil_run_noalloc(prob, opts, plan, nsweeps, stream.cuda_stream, rep)
        assert s == abft.ABFT_OK, abft.abft_last_error(None)
        g = (ut if nsweeps % 2 == 0 else u1).cpu().numpy()
    r, e = _as_dict(abft, rep, ev)
    return g, r, e


def test_two_calls_in_a_row_match_the_existing_entry_points(abft):
    import torch
    stream = torch.cuda.Stream()
    cases = [((16, 256, 512), 12, [(3, 7, 100, 511, 27), (8, 0, 0, 0, 29),
                                   (5, 9, 30, 200, 26, 0, W.FAULT_MEMORY)]),
             ((4, 64, 128), 9, [(2, 1, 63, 5, 30), (6, 3, 10, 127, 25)])]
    for shape, nsweeps, rows in cases:
        nz, ny, nx = shape
        u0, C = W.thermal_grid(nx, ny, nz, np.float32)
        plan = W.make_plan(rows)
        plan.sort(order="sweep", kind="stable")
        say("no-alloc", shape, nsweeps)
        g0, r0, e0 = _existing(abft, u0, C, plan, nsweeps, "online", True, stream)
        g1, r1, e1 = _noalloc(abft, u0, C, plan, nsweeps, "online", True, stream)
        assert np.array_equal(g0, g1), shape
        assert r0 == r1, (r0, r1)
        # the same events with the same values; blocks append them in any order
        key = ["sweep", "kind", "z", "y", "x", "a", "b"]
        assert np.array_equal(np.sort(e0, order=key), np.sort(e1, order=key))
        assert r1["corrected"] + r1["mem_corrected"] == len(rows)
        o, oev, _ = run_oracle(u0, W.THERMAL_TAPS, nsweeps, C=C, eps=1e-7, plan=plan)
        assert event_keys(e1) == event_keys(oev)
        assert_grid_close(g1, o, 1e-5, f"no-alloc {shape}")


def test_plain_mode_and_rejections(abft):
    import torch
    stream = torch.cuda.Stream()
    nz, ny, nx = 8, 96, 256
    u0, C = W.thermal_grid(nx, ny, nz, np.float32)
    say("no-alloc plain")
    g0, r0, _ = _existing(abft, u0, C, None, 7, "none", False, stream)
    g1, r1, e1 = _noalloc(abft, u0, C, None, 7, "none", False, stream)
    assert np.array_equal(g0, g1) and len(e1) == 0 and r1["sweeps_done"] == 7
    o, _, _ = run_oracle(u0, W.THERMAL_TAPS, 7, C=C, mode="none")
    assert_grid_close(g1, o, 1e-5, "no-alloc plain")
    # rejected before any device work: a workspace beyond the static array, offline mode,
    # an unsorted plan
    big = abft.make_problem((4096, 1024, 64), abft.ABFT_F32, W.THERMAL_TAPS, 0x1000, 0x2000)
    s = abft.abft_stencil_run_noalloc(big, abft.make_options("online"), None, 1, 0)
    assert s == abft.ABFT_E_UNSUPPORTED and "static scratch" in abft.abft_last_error(None)
    small = abft.make_problem((2, 8, 16), abft.ABFT_F32, W.THERMAL_TAPS, 0x1000, 0x2000)
    s = abft.abft_stencil_run_noalloc(small, abft.make_options("offline"), None, 1, 0)
    assert s == abft.ABFT_E_UNSUPPORTED
    unsorted = W.make_plan([(2, 0, 0, 0, 21), (5, 0, 0, 0, 20)])[::-1].copy()
    s = abft.abft_stencil_run_noalloc(small, abft.make_options("online"), unsorted, 6, 0)
    assert s == abft.ABFT_E_INVAL
