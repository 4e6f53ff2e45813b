/*
 * CPU oracle for ABFT-protected stencil sweeps
 * (Cavelan & Ciorba, "Algorithm-Based Fault Tolerance for Parallel Stencil Computations").
 *
 * TEST INFRASTRUCTURE ONLY.  This header and abft_oracle.c are the plain, slow reference
 * that the GPU library is checked against.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the library never includes, links or calls it.
 * It shares no code, header, table or constant with the GPU library.
 *
 * Grid layout: u[z][y][x], x fastest (the paper's index c = x + y*nx + z*nx*ny, Section 3.2).
 * Row checksum  B[z][y] = sum_x u[z][y][x]   (the paper's b_y, Eq.(3), computed every sweep)
 * Column checksum A[z][x] = sum_y u[z][y][x] (the paper's a_x, Eq.(2), computed on demand)
 */
#ifndef ABFT_ORACLE_H
#define ABFT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_F32 = 0, ORC_F64 = 1 };
enum { ORC_BC_CLAMP = 0, ORC_BC_PERIODIC = 1, ORC_BC_CONSTANT = 2 };
enum { ORC_MODE_NONE = 0, ORC_MODE_ONLINE = 1, ORC_MODE_OFFLINE = 2 };

/* Event kinds written by orc_run. */
enum {
    ORC_EV_ROW_FLAG = 1,       /* online row mismatch: sweep, z, y; a = direct, b = predicted */
    ORC_EV_CORRECTED = 2,      /* point corrected: sweep, z, y, x; a = old value, b = new value */
    ORC_EV_CHECKSUM_FAULT = 3, /* row flagged but no column flagged: sweep, z, y */
    ORC_EV_UNCORRECTABLE = 4,  /* >= 2 flagged rows and >= 2 flagged columns: sweep, z */
    ORC_EV_WINDOW_FLAG = 5,    /* offline row mismatch at window end: sweep, z, y, x = attempt */
    ORC_EV_ROLLBACK = 6,       /* offline rollback: sweep = window start, x = window length */
    ORC_EV_PERSISTENT = 7,     /* offline recompute still mismatched: sweep = window end */
    ORC_EV_COL_FLAG = 8,       /* column mismatch during location: sweep, z, x; a, b as above */
    ORC_EV_MEM_FLAG = 9,       /* input row of a sweep differs from its stored checksum:
                                  sweep, z, y; a = sum of the row as read, b = stored B */
    ORC_EV_MEM_CORRECTED = 10, /* input point repaired: sweep, z, y, x; a = old, b = new */
    ORC_EV_MEM_UNLOCATED = 11  /* input row mismatch that the weighted sums do not place:
                                  sweep, z, y; a = row sum difference, b = position ratio */
};

/* Fault kinds: a flip of the value a sweep stores (Section 5.1), or a flip of the sweep's
 * input grid in memory, after its checksums were taken and before the sweep reads it (the
 * first case of Theorem 2's proof). */
enum { ORC_FAULT_STORE = 0, ORC_FAULT_MEMORY = 1 };

typedef struct { int32_t dx, dy, dz, pad; double w; } orc_tap;

typedef struct {
    int64_t sweep;              /* STORE: sweep t whose stored output u^{t+1} is hit;
                                   MEMORY: sweep t whose input u^t is hit before it is read */
    int32_t z, y, x, bit, attempt, pad;
    int32_t kind;               /* ORC_FAULT_* */
    int32_t pad2;
} orc_fault;

typedef struct {
    int64_t sweep;
    int32_t kind, z, y, x;
    double a, b;
} orc_event;

typedef struct {
    int32_t nx, ny, nz;
    int32_t dtype;              /* storage type of u and C: ORC_F32 or ORC_F64 */
    int32_t ntaps;
    int32_t bc;                 /* ORC_BC_* */
    const orc_tap* taps;        /* weights are rounded to the storage type by the oracle */
    double bc_value;            /* ghost value for ORC_BC_CONSTANT */
    double c_scalar;            /* constant term when no C array is given */
} orc_problem;

typedef struct {
    int64_t sweeps_done;
    int64_t rows_flagged;       /* online row mismatches */
    int64_t cols_flagged;
    int64_t corrected;
    int64_t checksum_faults;
    int64_t uncorrectable;
    int64_t windows_checked;
    int64_t windows_flagged;
    int64_t rollbacks;
    int64_t persistent;
    int64_t events_total;       /* may exceed the event capacity */
    int64_t mem_flagged;        /* input rows that differed from their stored checksums */
    int64_t mem_corrected;
    int64_t mem_unlocated;
} orc_counters;

/* Returns 0 when the problem is valid, a negative code otherwise. */
int orc_validate(const orc_problem* p);

/* Eq.(1): uout = C + sum_S w * G(uin, x+dx, y+dy, z+dz), evaluated in double and rounded once
 * to the storage type.  C may be NULL (then p->c_scalar). */
void orc_sweep(const orc_problem* p, const void* C, const void* uin, void* uout);

/* Eq.(3) / Eq.(2), per layer, compensated double sums. */
void orc_row_checksums(const orc_problem* p, const void* u, double* B);
void orc_col_checksums(const orc_problem* p, const void* u, double* A);

/* Index-weighted row sums W[z][y] = sum_x (x + 1) u[z][y][x], compensated.  Together with
 * B they place a single changed point of a row: the change d moves B by d and W by
 * (x + 1) d. */
void orc_weighted_row_checksums(const orc_problem* p, const void* u, double* W);

/* Tile-local row checksums: the method applied on sub-domains (Section 3.1 defines the sweep
 * on a domain or sub-domain, chunk or block).  Each row is cut into tiles of T points
 * (T divides nx); Bt[z][y][k] = sum of u over tile k of row (z, y), compensated.  With C ==
 * NULL in orc_const_tile_checksums the scalar constant term is used. */
void orc_tile_checksums(const orc_problem* p, const void* u, int T, double* Bt);
void orc_const_tile_checksums(const orc_problem* p, const void* C, int T, double* cBt);

/* Theorem 1 for a tile as a sub-domain: the prediction of the next tile sums from the tile
 * sums of the input, the constant term's tile sums and the boundary terms of the tile, whose
 * ghost points are the neighbouring tiles' values inside the row and the boundary rule at
 * the row ends (read from the input grid uin).  Needs |dx| <= T for every tap. */
void orc_predict_tiles(const orc_problem* p, const double* cBt, const double* Bt,
                       const void* uin, int T, double* Bp);

/* The constant-term checksums c_y and c_x of Theorem 1. */
void orc_const_row_checksums(const orc_problem* p, const void* C, double* cB);
void orc_const_col_checksums(const orc_problem* p, const void* C, double* cA);

/* Boundary strips: for every row line (z, y) the first r and the last r values along x,
 * stored as 2*r doubles; r = orc_strip_width(p, axis).  Column lines likewise along y. */
int orc_strip_width(const orc_problem* p, int axis /* 0 = x (rows), 1 = y (columns) */);
void orc_row_strips(const orc_problem* p, const void* u, double* strips);
void orc_col_strips(const orc_problem* p, const void* u, double* strips);

/* Theorem 1, Eq.(5) (rows) and Eq.(4) (columns): predicted checksums of the next sweep from
 * the current checksums, the constant-term checksums and the boundary terms beta / alpha. */
void orc_predict_rows(const orc_problem* p, const double* cB, const double* Bt,
                      const double* row_strips, double* Bp);
void orc_predict_cols(const orc_problem* p, const double* cA, const double* At,
                      const double* col_strips, double* Ap);

/* Section 3.4: flag[i] = !(|direct - pred| <= eps * |pred|).  Returns the number flagged. */
int64_t orc_detect(int64_t n, const double* direct, const double* pred, double eps,
                   uint8_t* flags);

/* Whole run: nsweeps sweeps from u_a (u_b is scratch of the same size), protected in the given
 * mode (ORC_MODE_*), with the fault plan applied (STORE faults to stored values, MEMORY faults
 * to a sweep's input grid before it is read).  The final grid is left in u_a.  period is the
 * offline window length.  With auto_correct == 0 in offline mode the run stops after the first
 * flagged window (the checkpoint is still valid) and sweeps_done tells where.  Online with
 * ORC_INPUT_CHECK, each sweep also compares the sums of its input rows with the stored
 * checksums; a mismatched row is repaired before the sweep's own flags are examined (see
 * online_check).  With ORC_RECOMPUTE, located points are evaluated again instead of being
 * rebuilt from the checksums (see locate_correct_layer).  tile_x > 0 (online or no
 * protection, without ORC_INPUT_CHECK) keeps tile-local checksums of tile_x points instead of
 * whole-row checksums (see online_check_tiles); 0 keeps row checksums.  Offline, the
 * checkpoint is the window's first input in place, so a MEMORY fault on a window's first
 * sweep corrupts the checkpoint too.  Events are written up to max_events.  Returns 0 or a
 * negative code. */
/* Options of orc_run (flags). */
enum {
    ORC_INPUT_CHECK = 1, /* online: check each sweep's input rows against the stored checksums;
                            offline: before a rollback, check the checkpoint's rows against
                            its stored checksums and restore a changed point */
    ORC_RECOMPUTE = 2    /* online: correct a located point by evaluating it again from the
                            sweep's input (stencil locality) instead of Eq.(10) */
};

/* What a flip of the plan did, recorded when it was applied (one record per plan entry, in
 * plan order).  The sums are of the clean row and column through the point (Eq.(3), Eq.(2))
 * just before the flip, in the grid it lands in (the stored output for STORE, the input for
 * MEMORY).  The relative signal is the change the check that sees the flip measures against
 * the row checksum (Section 3.4): online |after - before| / |row_sum|; offline the change of
 * the row sums carried from the flip's sweep to the window's last sweep by the linear part of
 * Theorem 1 (the checksum plane stepped with the stencil weights, no constant term, no
 * boundary terms), largest over the rows, over |row_sum|.  The boundary terms of a change
 * vanish under the periodic rule and cancel under the clamp rule when the two x weights of
 * each (dy, dz) pair are equal, so the carried change is then exact; under the constant rule
 * it leaves out what the change loses through the row ends, which only a change within
 * (steps x radius) points of an x edge has.  A non-finite change gives an infinite signal. */
typedef struct {
    int32_t applied;   /* times the flip was applied */
    int32_t skipped;   /* 1 when the guard band (orc_guard) left it out */
    double before, after;
    double row_sum, col_sum;
    double signal;     /* row signal as above */
    double col_signal; /* |after - before| / |col_sum| */
} orc_fault_info;

/* Test harness option of orc_run.  Where a flip's relative signal lies close to the
 * threshold, two correct implementations may decide differently under rounding (the direct
 * and predicted checksums each carry rounding noise).  A STORE flip on attempt 0 whose row
 * signal lies in [lo, hi], or (online) whose row signal is above hi and column signal in
 * [lo, hi], is then left out (not applied, skipped = 1), so that the run equals the run of
 * the plan without it.  lo > hi leaves every flip in.  info may be NULL. */
typedef struct {
    double lo, hi;
    orc_fault_info* info;
} orc_guard;

int orc_run(const orc_problem* p, const void* C, int mode, int period, double eps,
            int auto_correct, int flags, int tile_x, void* u_a, void* u_b, int64_t nsweeps,
            const orc_fault* faults, int64_t nfaults,
            orc_event* events, int64_t max_events, orc_counters* counters,
            const orc_guard* guard /* may be NULL: every flip applied, nothing recorded */);

/* Thread control for the OpenMP loops (results do not depend on it). */
void orc_set_threads(int n);
int orc_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
