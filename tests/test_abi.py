"""The C-ABI library loads, exports every entry point its header declares, and agrees with the
Python binding on struct layouts.  Host-side argument validation is exercised without a GPU
(no call here reaches a HIP runtime function)."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "abft_stencil.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"\b(abft_[a-z_]+)\s*\(", src)))


def test_header_declares_and_library_exports(tmp_path):
    from paper_1909_00709_amd import abft
    names = _declared()
    assert set(names) == set(abft.EXPORTED)
    lib = ctypes.CDLL(abft.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", abft.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}$", out, re.M), n


def test_struct_layouts_match_c(tmp_path):
    from paper_1909_00709_amd import abft
    prog = tmp_path / "layout.c"
    prog.write_text(r"""
#include <stddef.h>
#include <stdio.h>
#include "abft_stencil.h"
#define P(T, F) printf(#T "." #F " %zu\n", offsetof(T, F));
int main(void) {
  printf("abft_tap %zu\nabft_problem %zu\nabft_options %zu\nabft_event %zu\n"
         "abft_fault %zu\nabft_report %zu\n", sizeof(abft_tap), sizeof(abft_problem),
         sizeof(abft_options), sizeof(abft_event), sizeof(abft_fault), sizeof(abft_report));
  P(abft_problem, taps) P(abft_problem, bc_value) P(abft_problem, cterm)
  P(abft_problem, cterm_scalar) P(abft_problem, u0) P(abft_problem, u1) P(abft_problem, u2)
  P(abft_options, threshold) P(abft_options, csum) P(abft_options, tuning_cache)
  P(abft_options, input_check) P(abft_options, correction)
  P(abft_event, a) P(abft_event, grid) P(abft_fault, grid)
  P(abft_report, max_noise) P(abft_report, nevents) P(abft_report, events)
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(prog), "-o", str(exe)],
                   check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True,
                                                      text=True, check=True).stdout.splitlines())
    py = {"abft_tap": abft.AbftTap, "abft_problem": abft.AbftProblem,
          "abft_options": abft.AbftOptions, "abft_event": abft.AbftEvent,
          "abft_fault": abft.AbftFault, "abft_report": abft.AbftReport}
    for k, v in got.items():
        if "." in k:
            t, f = k.split(".")
            assert getattr(py[t], f).offset == int(v), k
        else:
            assert ctypes.sizeof(py[k]) == int(v), k
    import workloads
    assert workloads.FAULT_DTYPE.itemsize == int(got["abft_fault"])


def test_strerror_and_host_validation():
    from paper_1909_00709_amd import abft
    assert abft.abft_strerror(abft.ABFT_OK) == "ok"
    assert "could not be corrected" in abft.abft_strerror(abft.ABFT_E_UNCORRECTABLE)
    assert abft.abft_strerror(12345) == "unknown status"
    # argument checks that fail before any device call
    opts = abft.make_options("online", threshold=1e-7)
    taps = [(0, 0, 0, 0.5), (1, 0, 0, 0.25), (-1, 0, 0, 0.25)]
    bad = [
        abft.make_problem((0, 4, 4), abft.ABFT_F32, taps, 0x1000, 0x2000),      # nz = 0
        abft.make_problem((1, 4, 4), 7, taps, 0x1000, 0x2000),                  # dtype
        abft.make_problem((1, 4, 4), abft.ABFT_F32, taps, 0x1000, 0x1000),      # u0 == u1
        abft.make_problem((1, 4, 4), abft.ABFT_F32, taps, None, 0x2000),        # u0 NULL
        abft.make_problem((1, 4, 4), abft.ABFT_F32, taps, 0x1000, 0x2000, bc=9),
    ]
    for p in bad:
        s, ctx = abft.abft_stencil_init(p, opts, 0)
        assert s == abft.ABFT_E_INVAL and not ctx.value
        assert abft.abft_last_error(None) != ""
    good = abft.make_problem((1, 4, 4), abft.ABFT_F32, taps, 0x1000, 0x2000)
    for o in (abft.make_options("online", threshold=0.0),
              abft.make_options("offline", period=0, threshold=1e-7),
              abft.make_options("online", threshold=1e-7, csum=5),
              abft.make_options("online", threshold=float("nan"))):
        s, ctx = abft.abft_stencil_init(good, o, 0)
        assert s == abft.ABFT_E_INVAL and not ctx.value
    f64 = abft.make_problem((1, 4, 4), abft.ABFT_F64, taps, 0x1000, 0x2000)
    s, _ = abft.abft_stencil_init(f64, abft.make_options("online", csum="f32comp"), 0)
    assert s == abft.ABFT_E_INVAL
    s, _ = abft.abft_stencil_init(good, abft.make_options("offline", period=129), 0)
    assert s == abft.ABFT_E_UNSUPPORTED
    # null context is rejected, destroy(NULL) is a no-op
    assert abft.abft_stencil_step(None, 1) == abft.ABFT_E_INVAL
    assert abft.abft_stencil_check(None) == abft.ABFT_E_INVAL
    abft.abft_stencil_destroy(None)


def test_no_oracle_in_product():
    """The product package never refers to the oracle."""
    pkg = os.path.join(ROOT, "paper_1909_00709_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.lower(), f
