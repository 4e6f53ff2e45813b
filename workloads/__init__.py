"""Seeded synthetic inputs shared by the CPU oracle tests, the GPU tests and the benchmark.

This module only draws random numbers and lays them out; it holds none of the ABFT
method's arithmetic (no sweep, no checksum, no prediction).  Every array is generated
on the host in float64 with ``numpy.random.default_rng(seed)`` (PCG64) and then cast to
the grid dtype, so the oracle and the GPU path start from the same bits.

Grid layout everywhere is ``u[z][y][x]`` (C order, x fastest), the paper's linear index
``c = x + y*nx + z*nx*ny`` (Section 3.2, sweep listing).

The workloads stand in for the paper's HotSpot3D runs (Section 5.1), whose input files
are not available: same stencil form (7-point thermal update with a power/ambient
constant term), same tile shapes as Table 1 where they apply, synthetic values.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# --------------------------------------------------------------------------------------
# Fault plan record: one bit flip, applied to the value a sweep stores (Section 5.1), or to
# a sweep's input grid in memory before the sweep reads it.
# Layout (40 bytes) is part of the C interface of both the library and the oracle.
# --------------------------------------------------------------------------------------
FAULT_STORE, FAULT_MEMORY = 0, 1
FAULT_DTYPE = np.dtype([
    ("sweep", "<i8"),    # 0-based sweep index t; STORE hits u^{t+1}, MEMORY hits u^t
    ("z", "<i4"), ("y", "<i4"), ("x", "<i4"),
    ("bit", "<i4"),      # bit position in the stored word (0 = LSB)
    ("attempt", "<i4"),  # fires only on this attempt (0 = first run, 1 = offline recompute)
    ("grid", "<i4"),     # grid index in a batch of grids (0 for a single grid)
    ("kind", "<i4"),     # FAULT_STORE or FAULT_MEMORY
    ("pad", "<i4"),
])

# --------------------------------------------------------------------------------------
# Stencil definitions: taps are (dx, dy, dz, w), the paper's set S of Eq.(1).
# --------------------------------------------------------------------------------------
# 7-point thermal diffusion (HotSpot3D form).  cc_amb is the ambient coupling weight;
# "coefficients sum to 1" counts it with the seven grid weights: cc = 1 - 4*0.1 - 2*0.05 - 0.05.
THERMAL_W_NSEW = 0.1
THERMAL_W_UD = 0.05
THERMAL_CC_AMB = 0.05
THERMAL_T_AMB = 80.0
THERMAL_P_SCALE = 1e-3
THERMAL_CC = 1.0 - 4 * THERMAL_W_NSEW - 2 * THERMAL_W_UD - THERMAL_CC_AMB  # 0.45

THERMAL_TAPS = (
    (0, 0, 0, THERMAL_CC),
    (-1, 0, 0, THERMAL_W_NSEW), (1, 0, 0, THERMAL_W_NSEW),
    (0, -1, 0, THERMAL_W_NSEW), (0, 1, 0, THERMAL_W_NSEW),
    (0, 0, -1, THERMAL_W_UD), (0, 0, 1, THERMAL_W_UD),
)

# 2D 4-point average (the paper's example set S in Section 3.1), centre weight 0.
JACOBI_TAPS = (
    (0, -1, 0, 0.25), (-1, 0, 0, 0.25), (1, 0, 0, 0.25), (0, 1, 0, 0.25),
)

BC_CLAMP, BC_PERIODIC, BC_CONSTANT = 0, 1, 2
F32, F64 = 0, 1
NP_DTYPE = {F32: np.float32, F64: np.float64}


def thermal_grid(nx: int, ny: int, nz: int, dtype, seed_t: int = 0, seed_p: int = 1,
                 t_lo: float = 320.0, t_hi: float = 330.0, t_amb: float = THERMAL_T_AMB):
    """Initial temperature T0 = U[t_lo, t_hi) and constant term C = 1e-3*P + cc_amb*t_amb,
    P = U[0, 1).  C is folded once in float64 and rounded to the grid dtype."""
    rt = np.random.default_rng(seed_t)
    rp = np.random.default_rng(seed_p)
    t0 = t_lo + (t_hi - t_lo) * rt.random((nz, ny, nx))
    p = rp.random((nz, ny, nx))
    c = THERMAL_P_SCALE * p + THERMAL_CC_AMB * t_amb
    return t0.astype(dtype), c.astype(dtype)


def jacobi_grid(nx: int = 64, ny: int = 64, seed: int = 0):
    """U0 = U[0, 1) on a single layer (nz = 1), float64."""
    return np.random.default_rng(seed).random((1, ny, nx))


def empty_plan(n: int = 0) -> np.ndarray:
    return np.zeros(n, dtype=FAULT_DTYPE)


def make_plan(rows) -> np.ndarray:
    """rows: iterable of (sweep, z, y, x, bit[, attempt[, kind]])."""
    rows = list(rows)
    plan = empty_plan(len(rows))
    for i, r in enumerate(rows):
        plan[i]["sweep"], plan[i]["z"], plan[i]["y"], plan[i]["x"], plan[i]["bit"] = r[:5]
        plan[i]["attempt"] = r[5] if len(r) > 5 else 0
        plan[i]["kind"] = r[6] if len(r) > 6 else FAULT_STORE
    plan.sort(order="sweep", kind="stable")
    return plan


def random_plan(seed: int, nflips: int, nsweeps: int, shape, bits, distinct_sweeps=False,
                one_per_layer=True) -> np.ndarray:
    """nflips flips at uniform (sweep, z, y, x) with bit drawn from ``bits`` (a sequence).
    one_per_layer keeps at most one flip per (sweep, z); distinct_sweeps at most one per sweep."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    rows, used = [], set()
    while len(rows) < nflips:
        t = int(rng.integers(0, nsweeps))
        z = int(rng.integers(0, nz))
        y = int(rng.integers(0, ny))
        x = int(rng.integers(0, nx))
        b = int(bits[int(rng.integers(0, len(bits)))])
        key = t if distinct_sweeps else (t, z)
        if (distinct_sweeps or one_per_layer) and key in used:
            continue
        used.add(key)
        rows.append((t, z, y, x, b))
    return make_plan(rows)


# --------------------------------------------------------------------------------------
# The five workloads.
# --------------------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    dtype: int
    taps: tuple
    nsweeps: int
    bc: int = BC_CLAMP
    bc_value: float = 0.0
    eps: float = 1e-12
    mode: str = "online"
    period: int = 10
    extra: dict = field(default_factory=dict)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def npoints(self):
        return self.nx * self.ny * self.nz

    def inputs(self):
        """(u0, C) with C None when the constant term is zero."""
        if self.taps is JACOBI_TAPS:
            return jacobi_grid(self.nx, self.ny, seed=0), None
        return thermal_grid(self.nx, self.ny, self.nz, NP_DTYPE[self.dtype], 0, 1)


# C1: 2D Jacobi 64x64 fp64, 10 sweeps, online, one flip per run at bit 40..62.
C1 = Workload("jacobi2d_64x64_f64", 64, 64, 1, F64, JACOBI_TAPS, 10, eps=1e-12)
# C2: 3D thermal 512x512x8 fp64, 100 sweeps, online and offline (k = 10).
C2 = Workload("thermal3d_512x512x8_f64", 512, 512, 8, F64, THERMAL_TAPS, 100, eps=1e-12)
# C3: 3D thermal 512x512x64 fp32, 1000-flip campaign over bits 0..31.
C3 = Workload("thermal3d_512x512x64_f32", 512, 512, 64, F32, THERMAL_TAPS, 1000, eps=1e-7)
# C5: 3D thermal 1024x1024x128 fp32, 500 sweeps, offline every 10 sweeps, 50 flips.
# Offline threshold: on a smooth field the rounding of a row is coherent, up to half an ulp of
# the values per sweep (about 6e-8 of the row sum for fp32), and a window of k sweeps adds k
# of them before the comparison, so eps must exceed k * 6e-8.
C5 = Workload("thermal3d_1024x1024x128_f32", 1024, 1024, 128, F32, THERMAL_TAPS, 500,
              eps=1e-6, mode="offline", period=10)


def c1_plan(bit: int) -> np.ndarray:
    """One flip at (iteration, i=row y, j=column x) drawn from rng(1001); bit given."""
    rng = np.random.default_rng(1001)
    # draw the same site sequence for every bit, then pick the bit's own draw
    sites = [(int(rng.integers(0, C1.nsweeps)), int(rng.integers(0, C1.ny)),
              int(rng.integers(0, C1.nx))) for _ in range(63)]
    it, i, j = sites[bit]
    return make_plan([(it, 0, i, j, bit)])


def c2_plan(nflips: int) -> np.ndarray:
    return random_plan(1002 + nflips, nflips, C2.nsweeps, C2.shape, range(64))


def c3_campaign(nflips: int = 1000, nsweeps: int = 1000, shape=None) -> np.ndarray:
    """Sweep s gets one flip at bit s mod 32, at a site drawn from rng(1003)."""
    nz, ny, nx = shape or C3.shape
    rng = np.random.default_rng(1003)
    rows = []
    for s in range(nflips):
        rows.append((s % nsweeps, int(rng.integers(0, nz)), int(rng.integers(0, ny)),
                     int(rng.integers(0, nx)), s % 32))
    return make_plan(rows)


def c5_plan(nflips: int = 50) -> np.ndarray:
    return random_plan(1005, nflips, C5.nsweeps, C5.shape, range(32), distinct_sweeps=True)


# C4: 64 independent grids, nx, ny in {64, 80, ..., 256}, nz in [4, 32], fp32, 200 sweeps.
C4_NGRIDS = 64
C4_NSWEEPS = 200
C4_EPS = 1e-7


def c4_shapes(ngrids: int = C4_NGRIDS, seed: int = 4):
    rng = np.random.default_rng(seed)
    sizes = np.arange(64, 257, 16)
    out = []
    for _ in range(ngrids):
        nx = int(sizes[rng.integers(0, len(sizes))])
        ny = int(sizes[rng.integers(0, len(sizes))])
        nz = int(rng.integers(4, 33))
        out.append((nz, ny, nx))
    return out


def c4_inputs(shapes):
    """Per grid g: temperature seed 10+g, power seed 110+g."""
    return [thermal_grid(nx, ny, nz, np.float32, 10 + g, 110 + g)
            for g, (nz, ny, nx) in enumerate(shapes)]


def c4_plans(shapes, nsweeps: int = C4_NSWEEPS, nflipped: int = 8, seed: int = 1004):
    """One flip in each of ``nflipped`` distinct grids; returns {grid index: plan}."""
    rng = np.random.default_rng(seed)
    grids = rng.choice(len(shapes), size=min(nflipped, len(shapes)), replace=False)
    plans = {}
    for g in sorted(int(v) for v in grids):
        nz, ny, nx = shapes[g]
        plans[g] = make_plan([(int(rng.integers(0, nsweeps)), int(rng.integers(0, nz)),
                               int(rng.integers(0, ny)), int(rng.integers(0, nx)),
                               int(rng.integers(0, 32)))])
    return plans


def taps_array(taps) -> np.ndarray:
    """Taps as a structured array matching the C layout {int dx, dy, dz, pad; double w}."""
    dt = np.dtype([("dx", "<i4"), ("dy", "<i4"), ("dz", "<i4"), ("pad", "<i4"), ("w", "<f8")])
    a = np.zeros(len(taps), dtype=dt)
    for i, (dx, dy, dz, w) in enumerate(taps):
        a[i]["dx"], a[i]["dy"], a[i]["dz"], a[i]["w"] = dx, dy, dz, w
    return a
