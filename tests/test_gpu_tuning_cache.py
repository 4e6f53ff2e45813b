"""The autotuner's cache file: a tuned shape is written under a key that names the grid, the
mode and the kernel variant (stencil radius or box, input-side check, tile-local checksums),
read back by a new context of the same variant, and not used by another variant."""
import os
import tempfile

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import say
from tests.test_gpu_memory_faults import BOX, STAR2

pytestmark = pytest.mark.gpu

VARIANTS = [
    ("thermal", W.THERMAL_TAPS, dict()),
    ("thermal, input check", W.THERMAL_TAPS, dict(input_check=True)),
    ("thermal, tiles", W.THERMAL_TAPS, dict(tile_x=64)),
    ("radius 2", STAR2, dict()),
    ("box", BOX, dict()),
]


def test_cache_round_trip_per_variant():
    import torch
    from paper_1909_00709_amd import abft
    nz, ny, nx = 16, 96, 256
    u0, C = W.thermal_grid(nx, ny, nz, np.float32)
    fd, cache = tempfile.mkstemp(suffix=".tune")
    os.close(fd)
    try:
        tuned = {}
        for name, taps, kw in VARIANTS:
            say("tuning cache:", name)
            kw = dict(dict(input_check=False), **kw)
            S = abft.Stencil(torch.from_numpy(u0).cuda(), taps, C=torch.from_numpy(C).cuda(),
                             threshold=4e-7, tuning_cache=cache, **kw)
            S.autotune()
            tuned[name] = S.launch_shape()
            S.close()
        lines = [l.split() for l in open(cache) if l.strip()]
        assert len(lines) == len(VARIANTS)  # one line per variant, none overwritten
        for name, taps, kw in VARIANTS:
            kw = dict(dict(input_check=False), **kw)
            S = abft.Stencil(torch.from_numpy(u0).cuda(), taps, C=torch.from_numpy(C).cuda(),
                             threshold=4e-7, tuning_cache=cache, **kw)
            assert S.launch_shape() == tuned[name], name
            S.step(2)
            rep, _ = S.check()
            assert rep["rows_flagged"] == 0
            S.close()
    finally:
        os.unlink(cache)
