"""The C interface's contract (include/abft_stencil.h), on the GPU: exact status codes of calls
made in the wrong state, `step` returning before the enqueued sweeps finish (no host
synchronisation), the caller's buffers intact and usable after `destroy`, and the documented
capacity of one sweep's flag lists (1024 flagged rows, 64 flagged input rows), at and past the
limit, against the oracle, which has no such limit."""
import time

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import assert_grid_close, event_keys, run_gpu, run_oracle, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def abft():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    from paper_1909_00709_amd import abft as A
    return A


def test_state_errors_exact(abft):
    """Offline without auto-correct: after a flagged window, step is refused with
    ABFT_E_STATE (the window awaits correct), and so is autotune; graph steps are not
    offered offline (ABFT_E_UNSUPPORTED).  After correct, step runs again."""
    import torch
    nz, ny, nx = 4, 64, 128
    u0, C = W.thermal_grid(nx, ny, nz, np.float64)
    say("state errors")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        S = abft.Stencil(torch.from_numpy(u0).cuda(), W.THERMAL_TAPS,
                         C=torch.from_numpy(C).cuda(), mode="offline", period=5,
                         threshold=1e-12, auto_correct=False, stream=stream)
        try:
            with pytest.raises(abft.AbftError) as e:
                S.step_graph(5)
            assert e.value.status == abft.ABFT_E_UNSUPPORTED
            S.inject(W.make_plan([(7, 2, 10, 20, 58)]))
            S.step(10)
            rep, _ = S.check()
            assert rep["pending"] > 0
            assert abft.abft_stencil_step(S.ctx, 1) == abft.ABFT_E_STATE
            with pytest.raises(abft.AbftError) as e:
                S.step(1)
            assert e.value.status == abft.ABFT_E_STATE
            assert abft.abft_stencil_autotune(S.ctx) == abft.ABFT_E_STATE
            s, rep, _ = S.correct()
            assert s == abft.ABFT_OK and rep["pending"] == 0 and rep["rollbacks"] == 1
            assert abft.abft_stencil_step(S.ctx, 5) == abft.ABFT_OK
        finally:
            S.close()
    # a step with a negative count, and calls on a NULL context
    assert abft.abft_stencil_step(None, 1) == abft.ABFT_E_INVAL
    assert abft.abft_stencil_check(None) == abft.ABFT_E_INVAL


@pytest.mark.parametrize("mode", ["none", "online", "offline"])
def test_step_returns_before_the_sweeps_finish(abft, mode):
    """step enqueues and returns: on a 1024 x 1024 x 128 fp32 grid, 60 sweeps take some 16 ms
    of GPU time; the call returns long before the stream drains, and the stream is still busy
    when it does."""
    import torch
    shape = (128, 1024, 1024)
    say("no host sync", mode)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        u0 = 320 + 10 * torch.rand(shape, device="cuda", dtype=torch.float32)
        C = torch.full(shape, 4.0, device="cuda", dtype=torch.float32)
        S = abft.Stencil(u0, W.THERMAL_TAPS, C=C, mode=mode, period=10, threshold=1e-6,
                         stream=stream)
        try:
            S.step(20)  # first launches: kernel attributes set, code loaded
            S.check()
            stream.synchronize()
            t0 = time.perf_counter()
            S.step(60)
            t_call = time.perf_counter() - t0
            busy = not stream.query()
            stream.synchronize()
            t_all = time.perf_counter() - t0
            rep, _ = S.check()
        finally:
            S.close()
    print(f"{mode}: step returned after {t_call * 1e3:.2f} ms, sweeps done after "
          f"{t_all * 1e3:.2f} ms")
    assert busy
    assert t_call < 0.5 * t_all, (t_call, t_all)
    assert rep["sweeps_done"] == 80


def test_caller_buffers_after_destroy(abft):
    """destroy frees only the library's workspace: the caller's grid buffers and constant
    term keep their contents (the result of the run and the unchanged constant term) and
    stay usable by the caller; new allocations do not land on them."""
    import torch
    nz, ny, nx = 8, 96, 256
    u0, C = W.thermal_grid(nx, ny, nz, np.float32)
    say("buffers after destroy")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ut = torch.from_numpy(u0).cuda()
        Ct = torch.from_numpy(C).cuda()
        S = abft.Stencil(ut, W.THERMAL_TAPS, C=Ct, mode="offline", period=4, threshold=1e-6,
                         stream=stream)
        S.step(10)
        S.check()
        cur, t = S.current()
        before = cur.cpu().numpy().copy()
        bufs = list(S.bufs)
        S.close()
        junk = [torch.full((nz, ny, nx), -1.0, device="cuda") for _ in range(4)]
        stream.synchronize()
        assert np.array_equal(cur.cpu().numpy(), before)
        assert np.array_equal(Ct.cpu().numpy(), C)
        for b in bufs:
            b.mul_(1.0)  # still a live, writable device buffer
        assert float(cur.sum()) == pytest.approx(float(before.astype(np.float64).sum()),
                                                 rel=1e-6)
        del junk
    o, _, _ = run_oracle(u0, W.THERMAL_TAPS, 10, C=C, mode="offline", period=4, eps=1e-6)
    assert_grid_close(before, o, 1e-5, "offline run read after destroy")


def _one_flip_per_layer(nflips, kind=W.FAULT_STORE, bit=55):
    return W.make_plan([(2, z, z % 4, (7 * z) % 64, bit, 0, kind) for z in range(nflips)])


@pytest.mark.parametrize("nflips", [1024, 1025])
def test_flagged_row_capacity(nflips):
    """One sweep holds at most 1024 flagged rows for location.  With one flip in each of 1024
    layers every flip is located and corrected, as in the oracle; with 1025 the GPU reports
    the sweep uncorrectable (one event: layer -1, a = number of flagged rows) and leaves the
    grid as it is, while the oracle corrects all 1025."""
    shape = (1100, 4, 64)
    rng = np.random.default_rng(9)
    u0 = 1.0 + rng.random(shape)
    plan = _one_flip_per_layer(nflips)
    say("flag capacity", nflips)
    # the flips land in the last of three sweeps
    g, gev, grep, _ = run_gpu(u0, W.THERMAL_TAPS, 3, eps=1e-12, plan=plan, input_check=False,
                              max_events=1 << 14)
    o, oev, ocnt = run_oracle(u0, W.THERMAL_TAPS, 3, eps=1e-12, plan=plan, input_check=False)
    assert grep["rows_flagged"] == ocnt["rows_flagged"] == nflips
    assert ocnt["corrected"] == nflips and ocnt["uncorrectable"] == 0
    if nflips <= 1024:
        assert event_keys(gev) == event_keys(oev)
        assert_grid_close(g, o, 1e-12, "1024 flagged rows")
    else:
        assert grep["corrected"] == 0 and grep["uncorrectable"] == 1
        unc = gev[gev["kind"] == 4]
        assert len(unc) == 1 and unc[0]["z"] == -1 and unc[0]["a"] == nflips


@pytest.mark.parametrize("nflips", [64, 65])
def test_flagged_input_row_capacity(nflips):
    """With the input-side check one sweep holds at most 64 mismatched input rows for repair:
    64 memory flips in distinct layers are placed and repaired as in the oracle; 65 are
    reported as one uncorrectable event (layer -1, a = number of rows, b = 1) and the oracle
    repairs all 65."""
    shape = (80, 4, 64)
    rng = np.random.default_rng(10)
    u0 = 1.0 + rng.random(shape)
    plan = _one_flip_per_layer(nflips, kind=W.FAULT_MEMORY, bit=54)
    say("input flag capacity", nflips)
    # the flips land in the input of the last of three sweeps
    g, gev, grep, _ = run_gpu(u0, W.THERMAL_TAPS, 3, eps=1e-12, plan=plan, input_check=True,
                              max_events=1 << 14)
    o, oev, ocnt = run_oracle(u0, W.THERMAL_TAPS, 3, eps=1e-12, plan=plan, input_check=True)
    assert ocnt["mem_corrected"] == nflips
    if nflips <= 64:
        assert grep["mem_corrected"] == nflips
        assert event_keys(gev) == event_keys(oev)
        assert_grid_close(g, o, 1e-12, "64 input rows")
    else:
        assert grep["mem_corrected"] == 0 and grep["uncorrectable"] >= 1
        unc = gev[(gev["kind"] == 4) & (gev["b"] == 1.0)]
        assert len(unc) == 1 and unc[0]["z"] == -1 and unc[0]["a"] == nflips
