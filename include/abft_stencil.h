/*
 * abft_stencil.h: C interface of the MI355X (gfx950) library for ABFT-protected stencil sweeps
 * (Cavelan & Ciorba, "Algorithm-Based Fault Tolerance for Parallel Stencil Computations").
 *
 * The library applies an iterated stencil sweep to a 2D or 3D grid on the GPU and protects
 * it against silent data corruption with the paper's checksums:
 *   - Section 3.1, Eq.(1): the sweep u' = C + sum_S w * u(x+dx, y+dy, z+dz);
 *   - Section 3.2, Eq.(2)-(3): direct checksums of the output (per layer z: row checksums
 *     B[z][y] = sum over x, computed in the same pass as every protected sweep; column
 *     checksums A[z][x] = sum over y, computed only after a mismatch);
 *   - Section 3.3, Theorem 1, Eq.(4)-(5): predicted checksums, the stencil applied to the
 *     previous checksums plus boundary terms;
 *   - Section 3.4, Theorem 2: a row is flagged when !(|B - B'| <= eps * |B'|);
 *   - Section 3.5, Eq.(10): the flagged row and column intersect at the corrupted point,
 *     whose value is recovered from the checksums;
 *   - Section 4: offline mode, a comparison every `period` sweeps with the interpolation
 *     applied `period` times, and rollback to the last verified state on a mismatch.
 *
 * Grid layout: u[z][y][x], x fastest (index x + nx*(y + ny*z)), in the caller's device memory.
 * All pointers named "device" are HIP device pointers on the current device; all others are
 * host pointers.  No call takes or returns a framework type.
 *
 * Ownership: the caller owns the grid buffers, the constant-term buffer and the stream.  They
 * must stay allocated from init to destroy and must not be written by the caller in between.
 * The library owns only its workspace (checksum planes, event log, a third grid buffer in
 * offline mode) and frees it in destroy.  It never frees or reallocates caller memory.
 *
 * Errors: every call returns an abft_status; none aborts or throws.  The text of the last
 * error of a context is kept for abft_last_error.  A detected corruption is data, not an
 * error: check() returns ABFT_OK and fills the report.
 *
 * Threads: a context may be used from one host thread at a time.  Calls on one context are
 * ordered on its stream; calls that overlap on the same context race.
 */
#ifndef ABFT_STENCIL_H
#define ABFT_STENCIL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ABFT_OK = 0,
    ABFT_E_INVAL = -1,          /* bad argument (NULL, size, range, duplicate tap, ...) */
    ABFT_E_UNSUPPORTED = -2,    /* valid but not implemented on the GPU (e.g. radius > 1) */
    ABFT_E_NOMEM = -3,          /* device or host allocation failed */
    ABFT_E_HIP = -4,            /* a HIP runtime call failed; see abft_last_error */
    ABFT_E_STATE = -5,          /* call not allowed in the context's current state */
    ABFT_E_UNCORRECTABLE = -6   /* detection that cannot be located or repaired */
} abft_status;

typedef enum { ABFT_F32 = 0, ABFT_F64 = 1 } abft_dtype;

/* Boundary rules, Section 3.3 "Dealing with Boundary Conditions": clamp repeats the edge
 * point (the sweep listing of Section 3.2), periodic wraps, constant uses bc_value for every
 * point outside the grid (0 gives the "empty" boundary). */
typedef enum { ABFT_BC_CLAMP = 0, ABFT_BC_PERIODIC = 1, ABFT_BC_CONSTANT = 2 } abft_bc;

/* NONE: plain sweeps (the unprotected baseline).  ONLINE: every sweep checked (Section 3).
 * OFFLINE: checked every `period` sweeps (Section 4). */
typedef enum { ABFT_MODE_NONE = 0, ABFT_MODE_ONLINE = 1, ABFT_MODE_OFFLINE = 2 } abft_mode;

/* Accumulation of the row checksums inside the sweep: fp64, or fp32 with compensated
 * (two-sum) accumulation.  Both are compared in fp64. */
typedef enum { ABFT_CSUM_F64 = 0, ABFT_CSUM_F32_COMP = 1 } abft_csum;

/* How an online correction rebuilds a located point (Section 3.5). */
typedef enum {
    ABFT_CORRECT_CHECKSUM = 0,  /* Eq.(10): from the row or column checksum and the other
                                   points of the line; rounding-limited; two or more rows and
                                   columns flagged in one layer are uncorrectable */
    ABFT_CORRECT_RECOMPUTE = 1  /* the point evaluated again from the sweep's input (which an
                                   online sweep leaves intact), exactly as the sweep computes
                                   it: bitwise the fault-free value; with several rows and
                                   columns flagged in a layer every intersection is evaluated
                                   again (at most 65536 per layer), unchanged points keep
                                   their value */
} abft_correction;

/* One stencil point of the set S of Eq.(1): offsets and weight.  The weight is rounded once
 * to the grid dtype; the sweep and the checksum prediction both use that rounded value. */
typedef struct {
    int32_t dx, dy, dz, pad;
    double w;
} abft_tap;

typedef struct {
    int32_t nx, ny, nz;         /* grid extents, >= 1 each; nz = 1 for a 2D grid */
    int32_t dtype;              /* abft_dtype of u0, u1 and cterm */
    int32_t ntaps;              /* number of taps, 1..27 on the GPU */
    int32_t bc;                 /* abft_bc */
    const abft_tap* taps;       /* host array of ntaps taps, copied by init.  GPU support:
                                   each offset at most once, either in the star of radius 2
                                   (the centre and points at distance 1 or 2 along one axis;
                                   an axis carrying a distance-2 tap must be at least 2 long)
                                   or in the 3 x 3 x 3 box (every offset in -1..1 per axis,
                                   diagonal taps included).  All grids of a batch
                                   (abft_stencil_init_batch) share the form: radius-1 star,
                                   radius-2 star or box. */
    double bc_value;            /* ghost value for ABFT_BC_CONSTANT, rounded to dtype */
    const void* cterm;          /* device [nz][ny][nx] constant term C of Eq.(1), or NULL */
    double cterm_scalar;        /* constant term used when cterm is NULL, rounded to dtype */
    void* u0;                   /* device grid; holds u^0 at init */
    void* u1;                   /* device grid of the same size; scratch, overwritten */
    void* u2;                   /* offline mode only: a third device grid of the same size for
                                   the checkpoint rotation, or NULL to let the library allocate
                                   it; ignored in the other modes */
} abft_problem;

typedef struct {
    int32_t mode;               /* abft_mode */
    int32_t period;             /* offline window length (sweeps per check), 1..128 */
    double threshold;           /* relative detection threshold eps of Section 3.4, > 0 */
    int32_t csum;               /* abft_csum */
    int32_t auto_correct;       /* 1: locate and correct (online) or roll back and recompute
                                   (offline) on the device without a host sync; 0: detection
                                   only, repair on abft_stencil_correct */
    int32_t max_events;         /* device event log capacity; 0 selects 4096 */
    int32_t input_check;        /* online (single grids and batches): 1 also checks each
                                   sweep's input rows
                                   against the checksums stored when they were written (the
                                   first case in the proof of Theorem 2, faults that arise in
                                   memory between sweeps) and, with auto_correct, repairs a
                                   changed input point and the outputs that read it; keeps an
                                   index-weighted row sum beside each checksum.  0: off.
                                   Ignored in the other modes. */
    const char* tuning_cache;   /* autotuner cache file (read at init, written by autotune),
                                   or NULL */
    int32_t correction;         /* an abft_correction value; online contexts and batches */
    int32_t tile_x;             /* 0: one checksum per row (Eq.(3)).  T > 0: tile-local
                                   checksums, the method applied on sub-domains of T points
                                   along x (Section 3.1's domain or sub-domain): one checksum
                                   per tile of each row, predicted by Theorem 1 on the tile
                                   with the neighbouring tiles as ghosts; errors in different
                                   tiles of one layer are located separately and a change is
                                   measured against a shorter sum.  On the GPU: online or
                                   unprotected single grids, star stencils, fp64 checksum
                                   accumulation, no input_check, T = 64 for fp32 grids and 32
                                   for fp64 grids, nx a multiple of T; otherwise
                                   ABFT_E_UNSUPPORTED. */
} abft_options;

/* Event kinds in the device log. */
enum {
    ABFT_EV_ROW_FLAG = 1,       /* online row mismatch: sweep, z, y; a = direct B, b = B' */
    ABFT_EV_CORRECTED = 2,      /* point repaired: sweep, z, y, x; a = old value, b = new */
    ABFT_EV_CHECKSUM_FAULT = 3, /* row flagged, no column flagged: checksum-side mismatch */
    ABFT_EV_UNCORRECTABLE = 4,  /* >= 2 rows and >= 2 columns flagged in a layer: sweep, z;
                                   a = rows, b = columns */
    ABFT_EV_WINDOW_FLAG = 5,    /* offline mismatch: sweep = last sweep of the window, z, y,
                                   x = attempt (0 first run, 1 recompute); a = B, b = B' */
    ABFT_EV_ROLLBACK = 6,       /* offline rollback: sweep = first sweep of the window,
                                   x = window length */
    ABFT_EV_PERSISTENT = 7,     /* offline recompute mismatched again: sweep = window end */
    ABFT_EV_COL_FLAG = 8,       /* column mismatch found while locating: sweep, z, x */
    ABFT_EV_MEM_FLAG = 9,       /* online: an input row of the sweep differs from the checksum
                                   stored when it was written: sweep, z, y; a = the row's sum
                                   as read, b = the stored B */
    ABFT_EV_MEM_CORRECTED = 10, /* input point repaired in place: sweep, z, y, x; a = old
                                   value, b = new; the sweep's outputs that read it are
                                   evaluated again */
    ABFT_EV_MEM_UNLOCATED = 11  /* input row mismatch that the weighted row sums do not place
                                   on one point: sweep, z, y; a = change of the row sum,
                                   b = implied position + 1 */
};

typedef struct {
    int64_t sweep;
    int32_t kind, z, y, x;
    double a, b;
    int32_t grid;               /* grid index in a batch context, 0 otherwise */
    int32_t pad;
} abft_event;

/* Fault kinds. */
enum {
    ABFT_FAULT_STORE = 0,       /* the value sweep `sweep` stores (Section 5.1 fault model) */
    ABFT_FAULT_MEMORY = 1       /* the input grid of sweep `sweep`, in memory, after its
                                   checksums were taken and before the sweep reads it (the
                                   first case in the proof of Theorem 2) */
};

/* A bit flip for the fault plan: XOR (1 << bit) into the word at (x, y, z).  STORE: into the
 * value sweep `sweep` stores, after the update and before the store, so the stored value and
 * its checksum both see it; it fires on the given attempt (0 = first run, 1 = offline
 * recompute after a rollback).  MEMORY: into u^sweep before sweep `sweep` reads it, on the
 * first attempt only (attempt must be 0).  In offline mode the
 * checkpoint is the window's first input in place, so a MEMORY flip on a window's first sweep
 * also corrupts the checkpoint. */
typedef struct {
    int64_t sweep;
    int32_t z, y, x, bit, attempt;
    int32_t grid;               /* grid index in a batch context, 0 otherwise */
    int32_t kind;               /* ABFT_FAULT_* */
    int32_t pad;
} abft_fault;

typedef struct {
    int64_t sweeps_done;        /* sweeps applied to the current grid */
    int64_t rows_flagged;
    int64_t cols_flagged;
    int64_t corrected;
    int64_t checksum_faults;
    int64_t uncorrectable;
    int64_t windows_checked;
    int64_t windows_flagged;
    int64_t rollbacks;
    int64_t persistent;
    int64_t events_total;       /* events appended to the device log (may exceed capacity) */
    int64_t pending;            /* detections waiting for abft_stencil_correct */
    int64_t sweeps_skipped;     /* offline without auto-correct: sweeps not run after a
                                   flagged window (re-issue them after correct) */
    int64_t mem_flagged;        /* online: input rows that differed from their checksums */
    int64_t mem_corrected;      /* online: input points repaired in place */
    int64_t mem_unlocated;      /* online: input row mismatches not placed on one point */
    double max_noise;           /* largest |B - B'| / |B'| over unflagged rows so far */
    int32_t nevents;            /* events copied into `events` by check() */
    int32_t events_cap;         /* capacity of `events` (set by the caller) */
    abft_event* events;         /* host array owned by the caller, or NULL */
} abft_report;

typedef struct abft_ctx abft_ctx;

/* Creates a context for one grid.  Validates p and o, copies the taps, allocates the
 * workspace and enqueues on `hip_stream` (a hipStream_t, or NULL for the null stream) the
 * constant-term checksums (Theorem 1's c_y, c_x) and the checksums of u0.  Returns
 * ABFT_E_INVAL for bad arguments, ABFT_E_UNSUPPORTED for stencils the GPU kernels do not
 * cover, ABFT_E_NOMEM / ABFT_E_HIP on allocation or runtime failures (nothing is leaked).
 * On success *out is a new context; on failure *out is NULL. */
abft_status abft_stencil_init(const abft_problem* p, const abft_options* o, void* hip_stream,
                              abft_ctx** out);

/* Creates one context for n independent grids (same dtype, any sizes) that run together:
 * each step is one launch over all grids' tiles.  p[i] as in abft_stencil_init; the options
 * apply to all grids (ONLINE or NONE only). */
abft_status abft_stencil_init_batch(const abft_problem* p, int32_t n, const abft_options* o,
                                    void* hip_stream, abft_ctx** out);

/* Enqueues nsweeps sweeps on the context's stream and returns without waiting for them
 * (offline mode without auto-correct is the exception: it waits at each window end and stops
 * after the first flagged window).  What a sweep does by mode: NONE, Eq.(1) alone; ONLINE,
 * Section 3: Eq.(1) with the row checksums of Eq.(3) in the same pass, their prediction by
 * Theorem 1 (Eq.(5)) and the test of Section 3.4, then with auto-correct the location and
 * correction of Section 3.5 (Eq.(10)); OFFLINE, Section 4: sweeps without checks, and at each
 * window end the interpolation applied `period` times, one comparison, and with auto-correct
 * the rollback to the checkpoint and the recompute of the window.  nsweeps >= 0.  ABFT_E_STATE while a detection awaits
 * abft_stencil_correct.  Offline with auto-correct, every window end enqueues the check and a
 * rollback recompute that runs only when the check flagged a mismatch: one launch of at most
 * one block per free block slot of the device, whose blocks wait for each other between the
 * window's sweeps, so compute units held by other streams delay it. */
abft_status abft_stencil_step(abft_ctx* ctx, int64_t nsweeps);

/* Enqueues nsweeps sweeps as one captured HIP graph (built on first use for a given nsweeps,
 * then replayed).  Same semantics as abft_stencil_step (Section 3 per sweep: Eq.(1), Eq.(3),
 * Theorem 1, the test of Section 3.4, and Section 3.5's correction with auto-correct); the fault plan is fixed when the
 * graph is built.  Not available in offline mode without auto-correct. */
abft_status abft_stencil_step_graph(abft_ctx* ctx, int64_t nsweeps);

/* Waits for the stream and reports the detections of Section 3.4 (online: flagged rows,
 * located and corrected points; offline: flagged windows, rollbacks).  In offline mode a
 * partial window is checked first (Section 4's detection "after completion" of the run),
 * which also closes it.  `out` may be NULL.  Returns
 * ABFT_E_HIP if a rollback recompute gave up waiting for its blocks (about three seconds at
 * one barrier): the recomputed window is then not to be trusted; the barrier is reset. */
abft_status abft_stencil_check(abft_ctx* ctx, abft_report* out);

/* Acts on pending detections: online, locates and corrects the flagged rows of the last
 * sweep (Section 3.5: column checksums of the flagged layer, Eq.(2), their prediction,
 * Eq.(4), the intersection, and the value of Eq.(10)); offline, rolls back to the checkpoint,
 * recomputes the window and checks it again (Section 4).
 * Returns ABFT_E_UNCORRECTABLE when a point cannot be located or repaired (the grid is left
 * as it is), ABFT_OK otherwise (also when nothing is pending).  `inout` may be NULL. */
abft_status abft_stencil_correct(abft_ctx* ctx, abft_report* inout);

/* The device buffer holding the current grid u^t of Eq.(1) (buffers rotate: online and plain
 * runs alternate u0 and u1, offline windows rotate three buffers so that the checkpoint of
 * Section 4 is never copied) and the sweep count t.  For a
 * batch context `grid` selects the grid; it must be 0 otherwise. */
abft_status abft_stencil_current(abft_ctx* ctx, int32_t grid, void** dev_ptr, int64_t* sweep);

/* The device plane [nz][ny] of fp64 row checksums that the next sweep's prediction uses
 * ([nz][ny][nx / T] tile checksums with tile-local checksums of T points). */
abft_status abft_stencil_checksums(abft_ctx* ctx, int32_t grid, double** dev_ptr);

/* Replaces the fault plan (a test harness for Section 5.1's bit-flip injection).  The plan
 * is copied; n = 0 clears it.  Entries outside the grid or the word size give ABFT_E_INVAL. */
abft_status abft_stencil_inject(abft_ctx* ctx, const abft_fault* f, int32_t n);

/* Times the candidate launch shapes on this context's grid (reads u0's current contents,
 * writes only the scratch buffer) and keeps the fastest; writes the tuning cache if one was
 * named.  For a batch context it times per-size-class layouts: the timing sweeps alternate
 * each grid's two buffers as a run does, and the current grids, checksums and weighted sums
 * are restored afterwards (the other buffer of each grid is overwritten).  Waits for the
 * stream. */
abft_status abft_stencil_autotune(abft_ctx* ctx);

/* Frees the library's workspace.  NULL is allowed.  Waits for the context's stream. */
void abft_stencil_destroy(abft_ctx* ctx);

/* Bytes of the static device array abft_stencil_run_noalloc works in, on each GPU. */
#define ABFT_NOALLOC_SCRATCH_BYTES (16u * 1024u * 1024u)

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): abft_stencil_init, abft_stencil_inject,
 * abft_stencil_step(nsweeps) and abft_stencil_check in one call, for one grid in the ONLINE or
 * NONE mode, that calls no hipMalloc, hipFree or other allocating routine.  Its workspace
 * (checksum planes, constant-term checksums, flag slots, counters, event log and fault plan)
 * lies in a static device array of ABFT_NOALLOC_SCRATCH_BYTES, one per GPU the library runs
 * on, held until the process ends.
 *   p, o: as for abft_stencil_init (o->tuning_cache is not read; the launch shape is the
 *         default one, as init gives without a tuning cache); offline mode and tile_x != 0
 *         give ABFT_E_UNSUPPORTED.
 *   faults: host array of nfaults entries sorted by sweep (attempt 0), or NULL with
 *         nfaults = 0; an unsorted plan gives ABFT_E_INVAL.
 *   nsweeps >= 0.  The grid after nsweeps sweeps is in u0 when nsweeps is even, in u1 when
 *         it is odd.
 *   out: filled as by abft_stencil_check (may be NULL).  The call waits for the stream.
 * Errors as for init, step and check; ABFT_E_UNSUPPORTED when the workspace (24 bytes per row
 * of the grid, 40 with the input check, 8 per column of each layer, two flag slots of 33 KB,
 * the event log and the plan, each rounded up to 256 bytes) exceeds the array.  The text is
 * in abft_last_error(NULL).  Every call on a GPU works in that GPU's one array and leaves its
 * contents there (each call clears what must start at zero): calls that overlap on one GPU,
 * from other threads or on other streams, race. */
abft_status abft_stencil_run_noalloc(const abft_problem* p, const abft_options* o,
                                     const abft_fault* faults, int32_t nfaults, int64_t nsweeps,
                                     void* hip_stream, abft_report* out);

/* Static text for a status code. */
const char* abft_strerror(abft_status s);

/* Text of the context's last error ("" if none); valid until the next call on ctx.  With
 * ctx NULL, the last error of a failed init or abft_stencil_run_noalloc on this thread. */
const char* abft_last_error(const abft_ctx* ctx);

/* Launch shape currently used by the context: rows per block, planes per block and lanes
 * per row of the sweep kernel (for benchmarks and tests). */
abft_status abft_stencil_launch_shape(const abft_ctx* ctx, int32_t* rows_per_block,
                                      int32_t* planes_per_block, int32_t* lanes_per_row);

#ifdef __cplusplus
}
#endif
#endif /* ABFT_STENCIL_H */
