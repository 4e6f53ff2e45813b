/*
 * CPU oracle for ABFT-protected stencil sweeps
 * (Cavelan & Ciorba, "Algorithm-Based Fault Tolerance for Parallel Stencil Computations").
 *
 * TEST INFRASTRUCTURE ONLY: the reference the GPU library is checked against.  Only the tests,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares no code with
 * the GPU library.  Plain loops, no blocking or fusion; each function follows one step of the
 * paper and says which.  Floating point is double (fp64) throughout; grid values are stored in
 * the problem's storage type (float or double) exactly as the method stores them.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no fast-math: the compensated sums
 * rely on IEEE rounding).
 *
 * Parity pins: every function here is pinned by the CPU tests (library correlate for the sweep,
 * exactly rounded sums for the checksums, exact rational arithmetic for Theorem 1, closed forms
 * for whole runs, the paper's detectable-bit result for detection, rollback equality for the
 * offline mode).  No function is "parity unpinned".
 */
#include "abft_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------------------------
 * Storage access.  Values are read into double and written back rounded to the storage type.
 * ------------------------------------------------------------------------------------------ */
static double ld(int dtype, const void* u, int64_t i)
{
    return dtype == ORC_F32 ? (double)((const float*)u)[i] : ((const double*)u)[i];
}

static void st(int dtype, void* u, int64_t i, double v)
{
    if (dtype == ORC_F32)
        ((float*)u)[i] = (float)v;
    else
        ((double*)u)[i] = v;
}

static double round_to(int dtype, double v)
{
    return dtype == ORC_F32 ? (double)(float)v : v;
}

static size_t elem_size(int dtype) { return dtype == ORC_F32 ? 4 : 8; }

static int64_t idx(const orc_problem* p, int64_t x, int64_t y, int64_t z)
{
    return x + (int64_t)p->nx * (y + (int64_t)p->ny * z);
}

/* Boundary rules (Section 3.3, "Dealing with Boundary Conditions"): map one coordinate onto
 * [0, n).  Clamp repeats the edge point (the sweep listing of Section 3.2 uses the centre for
 * a missing neighbour), periodic wraps, and constant returns -1: the point is a ghost whose
 * value is the constant (zero gives the "empty" boundary). */
static int64_t map_coord(int bc, int64_t c, int64_t n)
{
    if (c >= 0 && c < n) return c;
    if (bc == ORC_BC_CLAMP) return c < 0 ? 0 : n - 1;
    if (bc == ORC_BC_PERIODIC) {
        int64_t m = c % n;
        return m < 0 ? m + n : m;
    }
    return -1;
}

/* G(u, x, y, z): the ghost-extended grid. */
static double ghost(const orc_problem* p, const void* u, int64_t x, int64_t y, int64_t z)
{
    int64_t mx = map_coord(p->bc, x, p->nx);
    int64_t my = map_coord(p->bc, y, p->ny);
    int64_t mz = map_coord(p->bc, z, p->nz);
    if (mx < 0 || my < 0 || mz < 0) return round_to(p->dtype, p->bc_value);
    return ld(p->dtype, u, idx(p, mx, my, mz));
}

/* ------------------------------------------------------------------------------------------
 * Compensated summation (Neumaier's improvement of Kahan summation).  Used for every checksum
 * so that the oracle's sums are the exact sums to within a few units of double rounding.
 * Non-finite partial sums fall back to the plain sum so that Inf stays Inf.
 * ------------------------------------------------------------------------------------------ */
typedef struct { double s, c; } csum;

static void cs_add(csum* a, double v)
{
    double t = a->s + v;
    if (isfinite(t)) {
        if (fabs(a->s) >= fabs(v))
            a->c += (a->s - t) + v;
        else
            a->c += (v - t) + a->s;
    }
    a->s = t;
}

static double cs_val(csum a) { return isfinite(a.s) ? a.s + a.c : a.s; }

/* ------------------------------------------------------------------------------------------ */
int orc_validate(const orc_problem* p)
{
    if (!p || p->nx < 1 || p->ny < 1 || p->nz < 1) return -1;
    if (p->dtype != ORC_F32 && p->dtype != ORC_F64) return -1;
    if (p->bc < ORC_BC_CLAMP || p->bc > ORC_BC_CONSTANT) return -1;
    if (p->ntaps < 0 || (p->ntaps > 0 && !p->taps)) return -1;
    for (int k = 0; k < p->ntaps; k++) {
        /* Theorem 1's boundary terms need the shift to stay within one line length. */
        if (abs(p->taps[k].dx) > p->nx || abs(p->taps[k].dy) > p->ny ||
            abs(p->taps[k].dz) > p->nz)
            return -2;
    }
    return 0;
}

static double* rounded_weights(const orc_problem* p)
{
    double* w = (double*)malloc(sizeof(double) * (size_t)(p->ntaps > 0 ? p->ntaps : 1));
    for (int k = 0; k < p->ntaps; k++) w[k] = round_to(p->dtype, p->taps[k].w);
    return w;
}

/* Eq.(1) at one point, before the rounding to the storage type: w are the rounded weights,
 * cs the rounded scalar constant term. */
static double point(const orc_problem* p, const double* w, double cs, const void* C,
                    const void* uin, int64_t x, int64_t y, int64_t z)
{
    double acc = C ? ld(p->dtype, C, idx(p, x, y, z)) : cs;
    for (int k = 0; k < p->ntaps; k++)
        acc += w[k] * ghost(p, uin, x + p->taps[k].dx, y + p->taps[k].dy, z + p->taps[k].dz);
    return acc;
}

/* Eq.(1), Section 3.1: out-of-place sweep. */
void orc_sweep(const orc_problem* p, const void* C, const void* uin, void* uout)
{
    double* w = rounded_weights(p);
    const double cs = round_to(p->dtype, p->c_scalar);
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t z = 0; z < p->nz; z++)
        for (int64_t y = 0; y < p->ny; y++)
            for (int64_t x = 0; x < p->nx; x++)
                st(p->dtype, uout, idx(p, x, y, z), point(p, w, cs, C, uin, x, y, z));
    free(w);
}

/* Eq.(3) per layer: B[z][y] = sum over x. */
void orc_row_checksums(const orc_problem* p, const void* u, double* B)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t z = 0; z < p->nz; z++)
        for (int64_t y = 0; y < p->ny; y++) {
            csum s = {0.0, 0.0};
            for (int64_t x = 0; x < p->nx; x++) cs_add(&s, ld(p->dtype, u, idx(p, x, y, z)));
            B[z * p->ny + y] = cs_val(s);
        }
}

/* Eq.(2) per layer: A[z][x] = sum over y. */
void orc_col_checksums(const orc_problem* p, const void* u, double* A)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t z = 0; z < p->nz; z++)
        for (int64_t x = 0; x < p->nx; x++) {
            csum s = {0.0, 0.0};
            for (int64_t y = 0; y < p->ny; y++) cs_add(&s, ld(p->dtype, u, idx(p, x, y, z)));
            A[z * p->nx + x] = cs_val(s);
        }
}

/* The index-weighted row sums (a location aid for changes of the stored grid; not part of
 * the paper's scheme). */
void orc_weighted_row_checksums(const orc_problem* p, const void* u, double* W)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t z = 0; z < p->nz; z++)
        for (int64_t y = 0; y < p->ny; y++) {
            csum s = {0.0, 0.0};
            for (int64_t x = 0; x < p->nx; x++)
                cs_add(&s, (double)(x + 1) * ld(p->dtype, u, idx(p, x, y, z)));
            W[z * p->ny + y] = cs_val(s);
        }
}

/* Tile-local row checksums (the method on sub-domains of T points along x). */
void orc_tile_checksums(const orc_problem* p, const void* u, int T, double* Bt)
{
    const int64_t ntx = p->nx / T;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t z = 0; z < p->nz; z++)
        for (int64_t y = 0; y < p->ny; y++)
            for (int64_t k = 0; k < ntx; k++) {
                csum s = {0.0, 0.0};
                for (int64_t x = k * T; x < (k + 1) * T; x++)
                    cs_add(&s, ld(p->dtype, u, idx(p, x, y, z)));
                Bt[(z * p->ny + y) * ntx + k] = cs_val(s);
            }
}

void orc_const_tile_checksums(const orc_problem* p, const void* C, int T, double* cBt)
{
    const double cs = round_to(p->dtype, p->c_scalar);
    const int64_t ntx = p->nx / T;
    for (int64_t z = 0; z < p->nz; z++)
        for (int64_t y = 0; y < p->ny; y++)
            for (int64_t k = 0; k < ntx; k++) {
                csum s = {0.0, 0.0};
                for (int64_t x = k * T; x < (k + 1) * T; x++)
                    cs_add(&s, C ? ld(p->dtype, C, idx(p, x, y, z)) : cs);
                cBt[(z * p->ny + y) * ntx + k] = cs_val(s);
            }
}

/* Boundary term of tile k of row (y, z) of u for a shift dx: the ghost points that enter the
 * tile minus the points that leave it.  Ghosts inside the row are the neighbouring tiles'
 * points; beyond the row ends the boundary rule applies (G). */
static double tile_boundary_term(const orc_problem* p, const void* u, int T, int64_t k,
                                 int64_t y, int64_t z, int dx)
{
    const int64_t x0 = k * T;
    double b = 0.0;
    if (dx > 0) {
        for (int q = 0; q < dx; q++)
            b += ghost(p, u, x0 + T + q, y, z) - ld(p->dtype, u, idx(p, x0 + q, y, z));
    } else if (dx < 0) {
        for (int q = 1; q <= -dx; q++)
            b += ghost(p, u, x0 - q, y, z) - ld(p->dtype, u, idx(p, x0 + T - q, y, z));
    }
    return b;
}

/* Theorem 1 on each tile: b'_{z,y,k} = c_{z,y,k} + sum_S w * (b_{z+dz, y+dy, k} + beta_k(dx)),
 * the shifted rows mapped by the boundary rule (a row of constant ghosts sums to T * g). */
void orc_predict_tiles(const orc_problem* p, const double* cBt, const double* Bt,
                       const void* uin, int T, double* Bp)
{
    double* w = rounded_weights(p);
    const double g = round_to(p->dtype, p->bc_value);
    const int64_t ntx = p->nx / T;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t z = 0; z < p->nz; z++)
        for (int64_t y = 0; y < p->ny; y++)
            for (int64_t k = 0; k < ntx; k++) {
                double acc = cBt[(z * p->ny + y) * ntx + k];
                for (int t = 0; t < p->ntaps; t++) {
                    const orc_tap* tp = &p->taps[t];
                    const int64_t yy = map_coord(p->bc, y + tp->dy, p->ny);
                    const int64_t zz = map_coord(p->bc, z + tp->dz, p->nz);
                    double R;
                    if (yy < 0 || zz < 0) {
                        R = (double)T * g;
                    } else {
                        R = Bt[(zz * p->ny + yy) * ntx + k];
                        if (tp->dx != 0) R += tile_boundary_term(p, uin, T, k, yy, zz, tp->dx);
                    }
                    acc += w[t] * R;
                }
                Bp[(z * p->ny + y) * ntx + k] = acc;
            }
    free(w);
}

/* c_y and c_x of Theorem 1: the checksums of the constant term, computed once. */
void orc_const_row_checksums(const orc_problem* p, const void* C, double* cB)
{
    const double cs = round_to(p->dtype, p->c_scalar);
    for (int64_t z = 0; z < p->nz; z++)
        for (int64_t y = 0; y < p->ny; y++) {
            csum s = {0.0, 0.0};
            for (int64_t x = 0; x < p->nx; x++)
                cs_add(&s, C ? ld(p->dtype, C, idx(p, x, y, z)) : cs);
            cB[z * p->ny + y] = cs_val(s);
        }
}

void orc_const_col_checksums(const orc_problem* p, const void* C, double* cA)
{
    const double cs = round_to(p->dtype, p->c_scalar);
    for (int64_t z = 0; z < p->nz; z++)
        for (int64_t x = 0; x < p->nx; x++) {
            csum s = {0.0, 0.0};
            for (int64_t y = 0; y < p->ny; y++)
                cs_add(&s, C ? ld(p->dtype, C, idx(p, x, y, z)) : cs);
            cA[z * p->nx + x] = cs_val(s);
        }
}

/* ------------------------------------------------------------------------------------------
 * Boundary strips.  Theorem 1's boundary terms only involve the first and last |shift| points
 * of a line, so the strips hold the first r and last r values of every line.
 * ------------------------------------------------------------------------------------------ */
int orc_strip_width(const orc_problem* p, int axis)
{
    int r = 0;
    for (int k = 0; k < p->ntaps; k++) {
        int d = axis == 0 ? abs(p->taps[k].dx) : abs(p->taps[k].dy);
        if (d > r) r = d;
    }
    return r;
}

void orc_row_strips(const orc_problem* p, const void* u, double* strips)
{
    const int r = orc_strip_width(p, 0);
    if (r == 0) return;
    for (int64_t z = 0; z < p->nz; z++)
        for (int64_t y = 0; y < p->ny; y++) {
            double* s = strips + (z * p->ny + y) * 2 * r;
            for (int i = 0; i < r; i++) {
                s[i] = ld(p->dtype, u, idx(p, i, y, z));
                s[r + i] = ld(p->dtype, u, idx(p, p->nx - r + i, y, z));
            }
        }
}

void orc_col_strips(const orc_problem* p, const void* u, double* strips)
{
    const int r = orc_strip_width(p, 1);
    if (r == 0) return;
    for (int64_t z = 0; z < p->nz; z++)
        for (int64_t x = 0; x < p->nx; x++) {
            double* s = strips + (z * p->nx + x) * 2 * r;
            for (int i = 0; i < r; i++) {
                s[i] = ld(p->dtype, u, idx(p, x, i, z));
                s[r + i] = ld(p->dtype, u, idx(p, x, p->ny - r + i, z));
            }
        }
}

/* Value at in-line position q (-r <= q < n + r) of one ghost-extended line of length n, read
 * from its strip s (first r values, then last r values). */
static double line_at(int bc, double g, const double* s, int r, int64_t n, int64_t q)
{
    if (q < 0) {
        if (bc == ORC_BC_CLAMP) return s[0];
        if (bc == ORC_BC_CONSTANT) return g;
        q += n; /* periodic */
    } else if (q >= n) {
        if (bc == ORC_BC_CLAMP) return s[2 * r - 1];
        if (bc == ORC_BC_CONSTANT) return g;
        q -= n;
    }
    if (q < r) return s[q];
    return s[r + (q - (n - r))];
}

/* Theorem 1's boundary term (beta for rows, alpha for columns), 0-based with exclusive upper
 * limits: shifting a line of length n by d changes its sum from sum_{q=0}^{n-1} to
 * sum_{q=d}^{n-1+d}; the difference is the d ghost points that enter minus the d points that
 * leave.  d > 0: sum_{q=n}^{n+d-1} G(q) - sum_{q=0}^{d-1} u(q);
 * d < 0: sum_{q=d}^{-1} G(q) - sum_{q=n+d}^{n-1} u(q). */
static double boundary_term(int bc, double g, const double* s, int r, int64_t n, int d)
{
    double beta = 0.0;
    if (d > 0) {
        for (int64_t q = n; q < n + d; q++) beta += line_at(bc, g, s, r, n, q);
        for (int64_t q = 0; q < d; q++) beta -= line_at(bc, g, s, r, n, q);
    } else if (d < 0) {
        for (int64_t q = d; q < 0; q++) beta += line_at(bc, g, s, r, n, q);
        for (int64_t q = n + d; q < n; q++) beta -= line_at(bc, g, s, r, n, q);
    }
    return beta;
}

/* Theorem 1, Eq.(5), for the per-layer row checksums of a 3D grid: the stencil applied to the
 * checksum plane, b'_{z,y} = c_{z,y} + sum_S w * (b_{z+dz, y+dy} + beta_{dx}(y+dy, z+dz)).
 * The summed axis (x) collapses and its shift is absorbed in beta; the other two axes keep
 * their shifts and their boundary rule.  A row that lies wholly in constant ghosts sums to
 * nx * g. */
void orc_predict_rows(const orc_problem* p, const double* cB, const double* Bt,
                      const double* row_strips, double* Bp)
{
    double* w = rounded_weights(p);
    const double g = round_to(p->dtype, p->bc_value);
    const int r = orc_strip_width(p, 0);
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t z = 0; z < p->nz; z++)
        for (int64_t y = 0; y < p->ny; y++) {
            double acc = cB[z * p->ny + y];
            for (int k = 0; k < p->ntaps; k++) {
                const orc_tap* t = &p->taps[k];
                int64_t yy = map_coord(p->bc, y + t->dy, p->ny);
                int64_t zz = map_coord(p->bc, z + t->dz, p->nz);
                double R;
                if (yy < 0 || zz < 0) {
                    R = (double)p->nx * g;
                } else {
                    const int64_t line = zz * p->ny + yy;
                    R = Bt[line];
                    if (t->dx != 0)
                        R += boundary_term(p->bc, g, row_strips + line * 2 * r, r, p->nx, t->dx);
                }
                acc += w[k] * R;
            }
            Bp[z * p->ny + y] = acc;
        }
    free(w);
}

/* Theorem 1, Eq.(4): the same for the column checksums, with x and y exchanged (alpha). */
void orc_predict_cols(const orc_problem* p, const double* cA, const double* At,
                      const double* col_strips, double* Ap)
{
    double* w = rounded_weights(p);
    const double g = round_to(p->dtype, p->bc_value);
    const int r = orc_strip_width(p, 1);
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t z = 0; z < p->nz; z++)
        for (int64_t x = 0; x < p->nx; x++) {
            double acc = cA[z * p->nx + x];
            for (int k = 0; k < p->ntaps; k++) {
                const orc_tap* t = &p->taps[k];
                int64_t xx = map_coord(p->bc, x + t->dx, p->nx);
                int64_t zz = map_coord(p->bc, z + t->dz, p->nz);
                double R;
                if (xx < 0 || zz < 0) {
                    R = (double)p->ny * g;
                } else {
                    const int64_t line = zz * p->nx + xx;
                    R = At[line];
                    if (t->dy != 0)
                        R += boundary_term(p->bc, g, col_strips + line * 2 * r, r, p->ny, t->dy);
                }
                acc += w[k] * R;
            }
            Ap[z * p->nx + x] = acc;
        }
    free(w);
}

/* Section 3.4: relative mismatch against the predicted checksum.  Written as a negated
 * "within tolerance" test so that NaN and Inf mismatches are flagged. */
int64_t orc_detect(int64_t n, const double* direct, const double* pred, double eps,
                   uint8_t* flags)
{
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; i++) {
        int f = !(fabs(direct[i] - pred[i]) <= eps * fabs(pred[i]));
        flags[i] = (uint8_t)f;
        cnt += f;
    }
    return cnt;
}

/* ------------------------------------------------------------------------------------------
 * Whole runs.
 * ------------------------------------------------------------------------------------------ */
typedef struct {
    const orc_problem* p;
    const void* C;
    double eps;
    int auto_correct;
    int input_check;
    int recompute;
    const orc_fault* faults;
    int64_t nfaults;
    orc_event* ev;
    int64_t ev_cap;
    orc_counters* cnt;
    /* work arrays */
    double *B, *Bn, *Bp, *cB, *cA, *At, *An, *Ap, *rs, *cs;
    uint8_t *rflag, *cflag;
    /* input-side check: weighted sums of u^t and u^{t+1}, sums of the input rows as read */
    double *W, *Wn, *Bi;
    uint8_t* mflag;
    double* w;       /* rounded weights */
    double c_scalar; /* rounded scalar constant term */
    int reach;       /* largest |offset| of any tap along any axis */
    int tile;        /* tile-local checksums of this many points, or 0 (whole rows) */
    int mode;        /* ORC_MODE_* */
    int64_t win_end; /* offline: last sweep of the current window */
    const orc_guard* guard;
} run_state;

static void emit(run_state* S, int64_t sweep, int kind, int z, int y, int x, double a, double b)
{
    if (S->cnt->events_total < S->ev_cap) {
        orc_event* e = &S->ev[S->cnt->events_total];
        e->sweep = sweep;
        e->kind = kind;
        e->z = z;
        e->y = y;
        e->x = x;
        e->a = a;
        e->b = b;
    }
    S->cnt->events_total++;
}

/* The value with one bit flipped (Section 5.1). */
static double flipped(int dtype, const void* u, int64_t i, int bit)
{
    if (dtype == ORC_F32) {
        uint32_t v;
        float f;
        memcpy(&v, (const float*)u + i, 4);
        v ^= (uint32_t)1u << bit;
        memcpy(&f, &v, 4);
        return (double)f;
    }
    uint64_t v;
    double d;
    memcpy(&v, (const double*)u + i, 8);
    v ^= (uint64_t)1u << bit;
    memcpy(&d, &v, 8);
    return d;
}

/* |change| / |sum|, infinite when either is not finite or the sum is zero. */
static double rel_signal(double change, double sum)
{
    const double r = fabs(change) / fabs(sum);
    return r <= 1.7976931348623157e308 ? r : INFINITY;
}

/* Offline: the change d of row (z, y) at sweep `sweep` carried to the window's last sweep by
 * the linear part of Theorem 1 (the stencil weights stepped on the checksum plane; a constant
 * ghost contributes nothing to a change), largest absolute entry over the plane. */
static double carried_change(const run_state* S, int z, int y, double d, int64_t steps)
{
    const orc_problem* p = S->p;
    const int64_t nrows = (int64_t)p->nz * p->ny;
    double* a = (double*)calloc((size_t)nrows, sizeof(double));
    double* b = (double*)calloc((size_t)nrows, sizeof(double));
    a[(int64_t)z * p->ny + y] = d;
    for (int64_t s = 0; s < steps; s++) {
        for (int64_t zz = 0; zz < p->nz; zz++)
            for (int64_t yy = 0; yy < p->ny; yy++) {
                double acc = 0.0;
                for (int k = 0; k < p->ntaps; k++) {
                    const int64_t my = map_coord(p->bc, yy + p->taps[k].dy, p->ny);
                    const int64_t mz = map_coord(p->bc, zz + p->taps[k].dz, p->nz);
                    if (my >= 0 && mz >= 0) acc += S->w[k] * a[mz * p->ny + my];
                }
                b[zz * p->ny + yy] = acc;
            }
        double* t = a;
        a = b;
        b = t;
    }
    double m = 0.0;
    for (int64_t l = 0; l < nrows; l++)
        if (!(fabs(a[l]) <= m)) m = fabs(a[l]);
    free(a);
    free(b);
    return m;
}

/* Records what flip F is about to do to grid u (orc_fault_info) and decides, under the guard
 * band, whether it is applied.  Returns 1 to apply it. */
static int guard_flip(run_state* S, int64_t f, const void* u, int64_t sweep, int attempt)
{
    const orc_problem* p = S->p;
    const orc_fault* F = &S->faults[f];
    const orc_guard* G = S->guard;
    const int64_t i = idx(p, F->x, F->y, F->z);
    const double before = ld(p->dtype, u, i), after = flipped(p->dtype, u, i, F->bit);
    csum rs = {0.0, 0.0}, cs = {0.0, 0.0};
    for (int64_t q = 0; q < p->nx; q++) cs_add(&rs, ld(p->dtype, u, idx(p, q, F->y, F->z)));
    for (int64_t q = 0; q < p->ny; q++) cs_add(&cs, ld(p->dtype, u, idx(p, F->x, q, F->z)));
    const double row = cs_val(rs), col = cs_val(cs), d = after - before;
    double sig = rel_signal(d, row);
    if (S->mode == ORC_MODE_OFFLINE && F->kind == ORC_FAULT_STORE && isfinite(sig) &&
        S->win_end > sweep)
        sig = rel_signal(carried_change(S, F->z, F->y, d, S->win_end - sweep), row);
    const double csig = rel_signal(d, col);
    int skip = 0;
    if (F->kind == ORC_FAULT_STORE && attempt == 0 && G->lo <= G->hi) {
        const int in_row = sig >= G->lo && sig <= G->hi;
        const int in_col = S->mode == ORC_MODE_ONLINE && sig > G->hi && csig >= G->lo &&
                           csig <= G->hi;
        skip = in_row || in_col;
    }
    if (G->info) {
        orc_fault_info* I = &G->info[f];
        if (I->applied == 0 && !I->skipped) {
            I->before = before;
            I->after = after;
            I->row_sum = row;
            I->col_sum = col;
            I->signal = sig;
            I->col_signal = csig;
        }
        if (skip)
            I->skipped = 1;
        else
            I->applied++;
    }
    return !skip;
}

/* Section 5.1 fault model: flip one bit of the value the sweep stores, after the update
 * (kind STORE, applied to uout), or of the sweep's input before it is read (kind MEMORY,
 * applied to uin). */
static void inject(run_state* S, void* uout, int64_t sweep, int attempt, int kind)
{
    const orc_problem* p = S->p;
    for (int64_t f = 0; f < S->nfaults; f++) {
        const orc_fault* F = &S->faults[f];
        if (F->sweep != sweep || F->attempt != attempt || F->kind != kind) continue;
        if (S->guard && !guard_flip(S, f, uout, sweep, attempt)) continue;
        const int64_t i = idx(p, F->x, F->y, F->z);
        if (p->dtype == ORC_F32) {
            uint32_t v;
            memcpy(&v, (float*)uout + i, 4);
            v ^= (uint32_t)1u << F->bit;
            memcpy((float*)uout + i, &v, 4);
        } else {
            uint64_t v;
            memcpy(&v, (double*)uout + i, 8);
            v ^= (uint64_t)1u << F->bit;
            memcpy((double*)uout + i, &v, 8);
        }
    }
}

/* Value implied by the row checksum for point (x, y, z): the predicted row sum minus the other
 * points of the row.  Eq.(10) written with the partial sum taken directly, which is the same
 * quantity without losing the row sum to a huge corrupted value. */
static double row_value(run_state* S, const void* u, int z, int y, int x)
{
    const orc_problem* p = S->p;
    csum s = {0.0, 0.0};
    for (int64_t q = 0; q < p->nx; q++)
        if (q != x) cs_add(&s, ld(p->dtype, u, idx(p, q, y, z)));
    return S->Bp[(int64_t)z * p->ny + y] - cs_val(s);
}

static double col_value(run_state* S, const void* u, int z, int y, int x)
{
    const orc_problem* p = S->p;
    csum s = {0.0, 0.0};
    for (int64_t q = 0; q < p->ny; q++)
        if (q != y) cs_add(&s, ld(p->dtype, u, idx(p, x, q, z)));
    return S->Ap[(int64_t)z * p->nx + x] - cs_val(s);
}

static void recompute_row(run_state* S, const void* u, int z, int y, double* B)
{
    const orc_problem* p = S->p;
    csum s = {0.0, 0.0};
    for (int64_t q = 0; q < p->nx; q++) cs_add(&s, ld(p->dtype, u, idx(p, q, y, z)));
    B[(int64_t)z * p->ny + y] = cs_val(s);
}

/* Most intersection points evaluated again in one layer (recompute correction). */
#define ORC_MAX_RECOMPUTE 65536

/* Sections 3.4-3.5 for one layer with flagged rows: the column checksums of the layer locate
 * the corrupted columns, the intersection gives the points, Eq.(10) gives their values.
 * With the recompute correction (the locality the paper cites for stencils: an output point
 * depends only on its stencil neighbours of the sweep's input, which is intact online) each
 * intersection point is evaluated again from the input; a point that was not corrupted gets
 * its own value back, so several rows and columns flagged together are corrected as well. */
static void locate_correct_layer(run_state* S, int64_t sweep, const void* uin, void* uout, int z)
{
    const orc_problem* p = S->p;
    int R = 0, K = 0;
    int* ys = (int*)malloc(sizeof(int) * (size_t)p->ny);
    int* xs = (int*)malloc(sizeof(int) * (size_t)p->nx);
    for (int y = 0; y < p->ny; y++)
        if (S->rflag[(int64_t)z * p->ny + y]) ys[R++] = y;
    for (int x = 0; x < p->nx; x++) {
        const int64_t l = (int64_t)z * p->nx + x;
        if (!(fabs(S->An[l] - S->Ap[l]) <= S->eps * fabs(S->Ap[l]))) {
            xs[K++] = x;
            S->cnt->cols_flagged++;
            emit(S, sweep, ORC_EV_COL_FLAG, z, -1, x, S->An[l], S->Ap[l]);
        }
    }
    if (K == 0) {
        /* Scenario 2 of the correction section: the grid is consistent with the other
         * direction, so the mismatch is in a checksum.  The stored row checksum is the direct
         * sum of the data, so nothing in the grid changes. */
        for (int i = 0; i < R; i++) {
            S->cnt->checksum_faults++;
            emit(S, sweep, ORC_EV_CHECKSUM_FAULT, z, ys[i], -1, S->Bn[(int64_t)z * p->ny + ys[i]],
                 S->Bp[(int64_t)z * p->ny + ys[i]]);
        }
    } else if (S->recompute && (int64_t)R * K <= ORC_MAX_RECOMPUTE) {
        for (int i = 0; i < R; i++)
            for (int j = 0; j < K; j++) {
                const int y = ys[i], x = xs[j];
                const int64_t c = idx(p, x, y, z);
                const double old = ld(p->dtype, uout, c);
                st(p->dtype, uout, c, point(p, S->w, S->c_scalar, S->C, uin, x, y, z));
                const double nv = ld(p->dtype, uout, c);
                if (memcmp(&old, &nv, sizeof(double)) != 0) { /* bits changed */
                    S->cnt->corrected++;
                    emit(S, sweep, ORC_EV_CORRECTED, z, y, x, old, nv);
                }
            }
        for (int i = 0; i < R; i++) recompute_row(S, uout, z, ys[i], S->Bn);
    } else if (R >= 2 && K >= 2) {
        S->cnt->uncorrectable++;
        emit(S, sweep, ORC_EV_UNCORRECTABLE, z, -1, -1, (double)R, (double)K);
    } else {
        for (int i = 0; i < R; i++)
            for (int j = 0; j < K; j++) {
                const int y = ys[i], x = xs[j];
                const int64_t c = idx(p, x, y, z);
                const double old = ld(p->dtype, uout, c);
                double v;
                if (R == 1 && K == 1)
                    v = 0.5 * (row_value(S, uout, z, y, x) + col_value(S, uout, z, y, x));
                else if (R == 1)
                    v = col_value(S, uout, z, y, x); /* one error per flagged column */
                else
                    v = row_value(S, uout, z, y, x); /* one error per flagged row */
                st(p->dtype, uout, c, v);
                S->cnt->corrected++;
                emit(S, sweep, ORC_EV_CORRECTED, z, y, x, old, ld(p->dtype, uout, c));
            }
        /* checksum update after correction */
        for (int i = 0; i < R; i++) recompute_row(S, uout, z, ys[i], S->Bn);
    }
    free(ys);
    free(xs);
}

/* Boundary rule for the outputs around a repaired input point: periodic wraps, the other
 * rules have no outputs outside the grid (a clamped read of an edge point comes from an output
 * inside the grid, which the window already holds). */
static int64_t window_coord(int bc, int64_t c, int64_t n)
{
    if (c >= 0 && c < n) return c;
    return bc == ORC_BC_PERIODIC ? map_coord(bc, c, n) : -1;
}

/* A memory-resident change of input row (z, y) of sweep t, found because the row's sum as
 * read differs from the checksum B^t stored when the row was written (Theorem 2, first case):
 * the change d = sum - B^t moves the weighted sum by (x + 1) d, which places the point; its
 * value is recovered from B^t and the other points of the row (the partial-sum form used for
 * Eq.(10)); the outputs of sweep t that read it (the window of the stencil's reach around it)
 * are evaluated again, and the row checksums of the output rows in that window recomputed.
 * Returns 1 when the point was repaired. */
/* Places the single changed point of row (z, y) of u, whose sum read is `sum_read` against
 * the stored checksum B and weighted sum W, and restores it from B (the partial-sum form of
 * Eq.(10)).  Returns its x, or -1 (reported as unplaced). */
static int place_and_restore(run_state* S, int64_t sweep, void* u, int z, int y,
                             double sum_read, double B, double W)
{
    const orc_problem* p = S->p;
    csum ws = {0.0, 0.0};
    for (int64_t q = 0; q < p->nx; q++)
        cs_add(&ws, (double)(q + 1) * ld(p->dtype, u, idx(p, q, y, z)));
    const double d = sum_read - B;
    const double ratio = (cs_val(ws) - W) / d;
    const double pos = nearbyint(ratio);
    if (!isfinite(ratio) || fabs(ratio - pos) > 0.25 || pos < 1.0 || pos > (double)p->nx) {
        S->cnt->mem_unlocated++;
        emit(S, sweep, ORC_EV_MEM_UNLOCATED, z, y, -1, d, ratio);
        return -1;
    }
    const int x = (int)pos - 1;
    const int64_t c = idx(p, x, y, z);
    const double old = ld(p->dtype, u, c);
    csum rest = {0.0, 0.0};
    for (int64_t q = 0; q < p->nx; q++)
        if (q != x) cs_add(&rest, ld(p->dtype, u, idx(p, q, y, z)));
    st(p->dtype, u, c, B - cs_val(rest));
    S->cnt->mem_corrected++;
    emit(S, sweep, ORC_EV_MEM_CORRECTED, z, y, x, old, ld(p->dtype, u, c));
    return x;
}

/* Offline, before a rollback: the checkpoint's rows against the checksums stored when it was
 * formed; a changed point is placed with the weighted sums and restored in place, so that the
 * recompute starts from the checkpoint as it was written.  sweep = the window's first. */
static void verify_checkpoint(run_state* S, int64_t sweep, void* ckpt, const double* Bck,
                              const double* Wck)
{
    const orc_problem* p = S->p;
    const int64_t nrows = (int64_t)p->nz * p->ny;
    orc_row_checksums(p, ckpt, S->Bi);
    orc_detect(nrows, S->Bi, Bck, S->eps, S->mflag);
    for (int64_t l = 0; l < nrows; l++)
        if (S->mflag[l]) {
            const int z = (int)(l / p->ny), y = (int)(l % p->ny);
            S->cnt->mem_flagged++;
            emit(S, sweep, ORC_EV_MEM_FLAG, z, y, -1, S->Bi[l], Bck[l]);
            place_and_restore(S, sweep, ckpt, z, y, S->Bi[l], Bck[l], Wck[l]);
        }
}

static int repair_input_row(run_state* S, int64_t sweep, void* uin, void* uout, int z, int y)
{
    const orc_problem* p = S->p;
    const int64_t l = (int64_t)z * p->ny + y;
    const int x = place_and_restore(S, sweep, uin, z, y, S->Bi[l], S->B[l], S->W[l]);
    if (x < 0) return 0;
    const int R = S->reach;
    for (int oz = -R; oz <= R; oz++)
        for (int oy = -R; oy <= R; oy++) {
            const int64_t zz = window_coord(p->bc, z + oz, p->nz);
            const int64_t yy = window_coord(p->bc, y + oy, p->ny);
            if (zz < 0 || yy < 0) continue;
            for (int ox = -R; ox <= R; ox++) {
                const int64_t xx = window_coord(p->bc, x + ox, p->nx);
                if (xx < 0) continue;
                st(p->dtype, uout, idx(p, xx, yy, zz),
                   point(p, S->w, S->c_scalar, S->C, uin, xx, yy, zz));
            }
            recompute_row(S, uout, (int)zz, (int)yy, S->Bn);
        }
    return 1;
}

/* Online ABFT after sweep t (Figure 1 steps 2-3, then Section 3.5), with the input-side check:
 *   1. the output's row checksums, their prediction from B^t and the input's boundary strips,
 *      and the row flags (as the sweep reports them);
 *   2. the input rows as read against B^t; each mismatched row is repaired (repair_input_row);
 *   3. after a repair, the flagged rows are tested again against predictions from the repaired
 *      input, and only those still mismatched go on to location and correction. */
static void online_check(run_state* S, int64_t sweep, void* uin, void* uout)
{
    const orc_problem* p = S->p;
    const int64_t nrows = (int64_t)p->nz * p->ny;
    orc_row_checksums(p, uout, S->Bn);
    orc_row_strips(p, uin, S->rs);
    orc_predict_rows(p, S->cB, S->B, S->rs, S->Bp);
    int64_t nf = orc_detect(nrows, S->Bn, S->Bp, S->eps, S->rflag);
    for (int64_t l = 0; l < nrows; l++)
        if (S->rflag[l]) {
            S->cnt->rows_flagged++;
            emit(S, sweep, ORC_EV_ROW_FLAG, (int)(l / p->ny), (int)(l % p->ny), -1, S->Bn[l],
                 S->Bp[l]);
        }
    int64_t nm = 0;
    if (S->input_check) {
        orc_row_checksums(p, uin, S->Bi);
        nm = orc_detect(nrows, S->Bi, S->B, S->eps, S->mflag);
    }
    for (int64_t l = 0; l < nrows && nm > 0; l++)
        if (S->mflag[l]) {
            S->cnt->mem_flagged++;
            emit(S, sweep, ORC_EV_MEM_FLAG, (int)(l / p->ny), (int)(l % p->ny), -1, S->Bi[l],
                 S->B[l]);
        }
    if (!S->auto_correct) return;
    if (nm > 0) {
        int repaired = 0;
        for (int64_t l = 0; l < nrows; l++)
            if (S->mflag[l])
                repaired += repair_input_row(S, sweep, uin, uout, (int)(l / p->ny),
                                             (int)(l % p->ny));
        if (repaired) {
            orc_row_strips(p, uin, S->rs);
            orc_predict_rows(p, S->cB, S->B, S->rs, S->Bp);
            nf = 0;
            for (int64_t l = 0; l < nrows; l++) {
                if (!S->rflag[l]) continue;
                S->rflag[l] = !(fabs(S->Bn[l] - S->Bp[l]) <= S->eps * fabs(S->Bp[l]));
                nf += S->rflag[l];
            }
        }
    }
    if (nf == 0) return;
    /* the second checksum direction, only now that a mismatch was seen */
    orc_col_checksums(p, uin, S->At);
    orc_col_strips(p, uin, S->cs);
    orc_predict_cols(p, S->cA, S->At, S->cs, S->Ap);
    orc_col_checksums(p, uout, S->An);
    for (int z = 0; z < p->nz; z++) {
        int any = 0;
        for (int y = 0; y < p->ny && !any; y++) any = S->rflag[(int64_t)z * p->ny + y];
        if (any) locate_correct_layer(S, sweep, uin, uout, z);
    }
}

/* Value implied by tile checksum of the tile holding (x, y, z): the predicted tile sum minus
 * the tile's other points (the partial-sum form of Eq.(10) on the sub-domain). */
static double tile_value(run_state* S, const void* u, int z, int y, int x)
{
    const orc_problem* p = S->p;
    const int T = S->tile;
    const int64_t ntx = p->nx / T, k = x / T;
    csum s = {0.0, 0.0};
    for (int64_t q = k * T; q < (k + 1) * T; q++)
        if (q != x) cs_add(&s, ld(p->dtype, u, idx(p, q, y, z)));
    return S->Bp[((int64_t)z * p->ny + y) * ntx + k] - cs_val(s);
}

static void recompute_tile(run_state* S, const void* u, int z, int y, int64_t k)
{
    const orc_problem* p = S->p;
    const int T = S->tile;
    const int64_t ntx = p->nx / T;
    csum s = {0.0, 0.0};
    for (int64_t q = k * T; q < (k + 1) * T; q++) cs_add(&s, ld(p->dtype, u, idx(p, q, y, z)));
    S->Bn[((int64_t)z * p->ny + y) * ntx + k] = cs_val(s);
}

/* Sections 3.4-3.5 on the tiles of one layer: the layer's flagged columns (whole columns, as
 * for rows), and for each flagged tile the flagged columns inside its x range.  A flagged tile
 * with none is a checksum-side mismatch.  A candidate point alone in its tile takes the tile
 * checksum's value, alone in its column the column's, alone in both their mean (the row
 * scheme's single-row single-column case); a candidate shared both ways makes the layer
 * uncorrectable.  With the recompute correction every candidate is evaluated again. */
static void locate_correct_layer_tiles(run_state* S, int64_t sweep, const void* uin, void* uout,
                                       int z)
{
    const orc_problem* p = S->p;
    const int T = S->tile;
    const int64_t ntx = p->nx / T;
    int K = 0, nt = 0, nc = 0;
    int* xs = (int*)malloc(sizeof(int) * (size_t)p->nx);
    int64_t* ft = (int64_t*)malloc(sizeof(int64_t) * (size_t)(p->ny * ntx));
    int* cy = (int*)malloc(sizeof(int) * (size_t)(p->ny * ntx) * 4 + 16);
    int* cx = (int*)malloc(sizeof(int) * (size_t)(p->ny * ntx) * 4 + 16);
    int64_t cap = p->ny * ntx * 4 + 4;
    for (int x = 0; x < p->nx; x++) {
        const int64_t l = (int64_t)z * p->nx + x;
        if (!(fabs(S->An[l] - S->Ap[l]) <= S->eps * fabs(S->Ap[l]))) {
            xs[K++] = x;
            S->cnt->cols_flagged++;
            emit(S, sweep, ORC_EV_COL_FLAG, z, -1, x, S->An[l], S->Ap[l]);
        }
    }
    int overflow = 0;
    for (int64_t yk = 0; yk < p->ny * ntx; yk++) {
        const int64_t l = (int64_t)z * p->ny * ntx + yk;
        if (!S->rflag[l]) continue;
        ft[nt++] = yk;
        const int y = (int)(yk / ntx);
        const int64_t k = yk % ntx;
        int found = 0;
        for (int j = 0; j < K; j++)
            if (xs[j] / T == k) {
                if (nc >= cap) {
                    overflow = 1;
                    break;
                }
                cy[nc] = y;
                cx[nc] = xs[j];
                nc++;
                found = 1;
            }
        if (!found) {
            S->cnt->checksum_faults++;
            emit(S, sweep, ORC_EV_CHECKSUM_FAULT, z, y, (int)(k * T), S->Bn[l], S->Bp[l]);
        }
    }
    if (nc > 0 && (overflow || (S->recompute && nc > ORC_MAX_RECOMPUTE))) {
        S->cnt->uncorrectable++;
        emit(S, sweep, ORC_EV_UNCORRECTABLE, z, -1, -1, (double)nt, (double)K);
    } else if (nc > 0 && S->recompute) {
        for (int i = 0; i < nc; i++) {
            const int64_t c = idx(p, cx[i], cy[i], z);
            const double old = ld(p->dtype, uout, c);
            st(p->dtype, uout, c, point(p, S->w, S->c_scalar, S->C, uin, cx[i], cy[i], z));
            const double nv = ld(p->dtype, uout, c);
            if (memcmp(&old, &nv, sizeof(double)) != 0) {
                S->cnt->corrected++;
                emit(S, sweep, ORC_EV_CORRECTED, z, cy[i], cx[i], old, nv);
            }
        }
    } else if (nc > 0) {
        int ambiguous = 0;
        int* in_tile = (int*)calloc((size_t)nc, sizeof(int));
        int* in_col = (int*)calloc((size_t)nc, sizeof(int));
        for (int i = 0; i < nc; i++)
            for (int j = 0; j < nc; j++) {
                if (cy[j] == cy[i] && cx[j] / T == cx[i] / T) in_tile[i]++;
                if (cx[j] == cx[i]) in_col[i]++;
            }
        for (int i = 0; i < nc; i++) ambiguous |= in_tile[i] > 1 && in_col[i] > 1;
        if (ambiguous) {
            S->cnt->uncorrectable++;
            emit(S, sweep, ORC_EV_UNCORRECTABLE, z, -1, -1, (double)nt, (double)K);
        } else {
            double* v = (double*)malloc(sizeof(double) * (size_t)nc);
            for (int i = 0; i < nc; i++) {
                if (in_tile[i] == 1 && in_col[i] == 1)
                    v[i] = 0.5 * (tile_value(S, uout, z, cy[i], cx[i]) +
                                  col_value(S, uout, z, cy[i], cx[i]));
                else if (in_tile[i] == 1)
                    v[i] = tile_value(S, uout, z, cy[i], cx[i]);
                else
                    v[i] = col_value(S, uout, z, cy[i], cx[i]);
            }
            for (int i = 0; i < nc; i++) {
                const int64_t c = idx(p, cx[i], cy[i], z);
                const double old = ld(p->dtype, uout, c);
                st(p->dtype, uout, c, v[i]);
                S->cnt->corrected++;
                emit(S, sweep, ORC_EV_CORRECTED, z, cy[i], cx[i], old, ld(p->dtype, uout, c));
            }
            free(v);
        }
        free(in_tile);
        free(in_col);
    }
    /* checksum update of the flagged tiles */
    for (int i = 0; i < nt; i++) recompute_tile(S, uout, z, (int)(ft[i] / ntx), ft[i] % ntx);
    free(xs);
    free(ft);
    free(cy);
    free(cx);
}

/* Online ABFT with tile-local checksums: the tile sums of the output, their prediction
 * (Theorem 1 on each tile) and the tile flags; after a flag the column stage of the rows
 * scheme and the tile case analysis (locate_correct_layer_tiles). */
static void online_check_tiles(run_state* S, int64_t sweep, const void* uin, void* uout)
{
    const orc_problem* p = S->p;
    const int T = S->tile;
    const int64_t ntx = p->nx / T, ntiles = (int64_t)p->nz * p->ny * ntx;
    orc_tile_checksums(p, uout, T, S->Bn);
    orc_predict_tiles(p, S->cB, S->B, uin, T, S->Bp);
    const int64_t nf = orc_detect(ntiles, S->Bn, S->Bp, S->eps, S->rflag);
    for (int64_t l = 0; l < ntiles; l++)
        if (S->rflag[l]) {
            S->cnt->rows_flagged++;
            emit(S, sweep, ORC_EV_ROW_FLAG, (int)(l / (p->ny * ntx)), (int)((l / ntx) % p->ny),
                 (int)((l % ntx) * T), S->Bn[l], S->Bp[l]);
        }
    if (!S->auto_correct || nf == 0) return;
    orc_col_checksums(p, uin, S->At);
    orc_col_strips(p, uin, S->cs);
    orc_predict_cols(p, S->cA, S->At, S->cs, S->Ap);
    orc_col_checksums(p, uout, S->An);
    for (int z = 0; z < p->nz; z++) {
        int any = 0;
        for (int64_t yk = 0; yk < p->ny * ntx && !any; yk++)
            any = S->rflag[(int64_t)z * p->ny * ntx + yk];
        if (any) locate_correct_layer_tiles(S, sweep, uin, uout, z);
    }
}

int orc_run(const orc_problem* p, const void* C, int mode, int period, double eps,
            int auto_correct, int flags, int tile_x, void* u_a, void* u_b, int64_t nsweeps,
            const orc_fault* faults, int64_t nfaults,
            orc_event* events, int64_t max_events, orc_counters* counters,
            const orc_guard* guard)
{
    int rc = orc_validate(p);
    if (rc) return rc;
    if (!u_a || !u_b || !counters || nsweeps < 0) return -1;
    if (mode < ORC_MODE_NONE || mode > ORC_MODE_OFFLINE) return -1;
    if (mode == ORC_MODE_OFFLINE && period < 1) return -1;
    if (tile_x < 0 || (tile_x > 0 && (p->nx % tile_x != 0 || mode == ORC_MODE_OFFLINE ||
                                      (flags & ORC_INPUT_CHECK))))
        return -1;
    for (int k = 0; k < p->ntaps && tile_x > 0; k++)
        if (abs(p->taps[k].dx) > tile_x) return -2;
    const int bits = p->dtype == ORC_F32 ? 32 : 64;
    for (int64_t f = 0; f < nfaults; f++) {
        const orc_fault* F = &faults[f];
        if (F->x < 0 || F->x >= p->nx || F->y < 0 || F->y >= p->ny || F->z < 0 ||
            F->z >= p->nz || F->bit < 0 || F->bit >= bits ||
            (F->kind != ORC_FAULT_STORE && F->kind != ORC_FAULT_MEMORY))
            return -3;
    }
    memset(counters, 0, sizeof(*counters));

    const int64_t n = (int64_t)p->nx * p->ny * p->nz;
    /* checksum entries: rows, or tiles of rows */
    const int64_t nrows = (int64_t)p->nz * p->ny * (tile_x > 0 ? p->nx / tile_x : 1),
                  ncols = (int64_t)p->nz * p->nx;
    const size_t bytes = (size_t)n * elem_size(p->dtype);
    const int rx = orc_strip_width(p, 0), ry = orc_strip_width(p, 1);

    run_state S;
    memset(&S, 0, sizeof(S));
    S.p = p;
    S.C = C;
    S.eps = eps;
    S.auto_correct = auto_correct;
    S.input_check = (flags & ORC_INPUT_CHECK) && mode != ORC_MODE_NONE;
    S.recompute = (flags & ORC_RECOMPUTE) != 0;
    S.tile = tile_x;
    S.mode = mode;
    S.guard = guard;
    if (guard && guard->info) memset(guard->info, 0, sizeof(orc_fault_info) * (size_t)nfaults);
    S.faults = faults;
    S.nfaults = nfaults;
    S.ev = events;
    S.ev_cap = events ? max_events : 0;
    S.cnt = counters;
    S.B = (double*)calloc((size_t)nrows, sizeof(double));
    S.Bn = (double*)calloc((size_t)nrows, sizeof(double));
    S.Bp = (double*)calloc((size_t)nrows, sizeof(double));
    S.cB = (double*)calloc((size_t)nrows, sizeof(double));
    S.cA = (double*)calloc((size_t)ncols, sizeof(double));
    S.At = (double*)calloc((size_t)ncols, sizeof(double));
    S.An = (double*)calloc((size_t)ncols, sizeof(double));
    S.Ap = (double*)calloc((size_t)ncols, sizeof(double));
    S.rs = (double*)calloc((size_t)nrows * 2 * (rx ? rx : 1), sizeof(double));
    S.cs = (double*)calloc((size_t)ncols * 2 * (ry ? ry : 1), sizeof(double));
    S.rflag = (uint8_t*)calloc((size_t)nrows, 1);
    S.cflag = (uint8_t*)calloc((size_t)ncols, 1);
    S.W = (double*)calloc((size_t)nrows, sizeof(double));
    S.Wn = (double*)calloc((size_t)nrows, sizeof(double));
    S.Bi = (double*)calloc((size_t)nrows, sizeof(double));
    S.mflag = (uint8_t*)calloc((size_t)nrows, 1);
    S.w = rounded_weights(p);
    S.c_scalar = round_to(p->dtype, p->c_scalar);
    for (int k = 0; k < p->ntaps; k++) {
        const int m = abs(p->taps[k].dx) > abs(p->taps[k].dy) ? abs(p->taps[k].dx)
                                                               : abs(p->taps[k].dy);
        if (m > S.reach) S.reach = m;
        if (abs(p->taps[k].dz) > S.reach) S.reach = abs(p->taps[k].dz);
    }
    if (tile_x > 0)
        orc_const_tile_checksums(p, C, tile_x, S.cB);
    else
        orc_const_row_checksums(p, C, S.cB);
    orc_const_col_checksums(p, C, S.cA);

    void* uin = u_a;
    void* uout = u_b;

    if (mode != ORC_MODE_OFFLINE) {
        if (mode == ORC_MODE_ONLINE) {
            if (tile_x > 0)
                orc_tile_checksums(p, uin, tile_x, S.B);
            else
                orc_row_checksums(p, uin, S.B);
        }
        if (S.input_check) orc_weighted_row_checksums(p, uin, S.W);
        for (int64_t t = 0; t < nsweeps; t++) {
            inject(&S, uin, t, 0, ORC_FAULT_MEMORY);
            orc_sweep(p, C, uin, uout);
            inject(&S, uout, t, 0, ORC_FAULT_STORE);
            if (mode == ORC_MODE_ONLINE) {
                if (tile_x > 0)
                    online_check_tiles(&S, t, uin, uout);
                else
                    online_check(&S, t, uin, uout);
                /* the weighted sums of the output as it stands after any repair */
                if (S.input_check) orc_weighted_row_checksums(p, uout, S.Wn);
                double* tmp = S.B;
                S.B = S.Bn;
                S.Bn = tmp;
                tmp = S.W;
                S.W = S.Wn;
                S.Wn = tmp;
            }
            void* tu = uin;
            uin = uout;
            uout = tu;
            counters->sweeps_done = t + 1;
        }
        if (uin != u_a) memcpy(u_a, uin, bytes);
    } else {
        /* Section 4: offline detection every `period` sweeps with checkpoint / rollback.
         * The checkpoint is a copy of the grid and of its row checksums. */
        void* ckpt = malloc(bytes);
        double* Bck = (double*)malloc(sizeof(double) * (size_t)nrows);
        double* Wck = (double*)malloc(sizeof(double) * (size_t)nrows);  /* input check */
        double* hist = (double*)malloc(sizeof(double) * (size_t)nrows * 2 * (rx ? rx : 1) *
                                       (size_t)period);
        memcpy(ckpt, u_a, bytes);
        orc_row_checksums(p, u_a, Bck);
        if (S.input_check) orc_weighted_row_checksums(p, u_a, Wck);
        int64_t t0 = 0;
        while (t0 < nsweeps) {
            const int64_t k = (nsweeps - t0 < period) ? nsweeps - t0 : period;
            int attempt = 0;
            int halt = 0;
            S.win_end = t0 + k - 1;
            for (;;) {
                uin = u_a;
                uout = u_b;
                for (int64_t j = 0; j < k; j++) {
                    inject(&S, uin, t0 + j, attempt, ORC_FAULT_MEMORY);
                    /* the checkpoint is the window's first input in place */
                    if (j == 0) inject(&S, ckpt, t0, attempt, ORC_FAULT_MEMORY);
                    orc_row_strips(p, uin, hist + j * nrows * 2 * rx);
                    orc_sweep(p, C, uin, uout);
                    inject(&S, uout, t0 + j, attempt, ORC_FAULT_STORE);
                    void* tu = uin;
                    uin = uout;
                    uout = tu;
                }
                if (uin != u_a) memcpy(u_a, uin, bytes);
                /* direct checksums of the window's result */
                orc_row_checksums(p, u_a, S.Bn);
                /* the interpolation applied k times from the checkpoint's checksums */
                memcpy(S.B, Bck, sizeof(double) * (size_t)nrows);
                for (int64_t j = 0; j < k; j++) {
                    orc_predict_rows(p, S.cB, S.B, hist + j * nrows * 2 * rx, S.Bp);
                    memcpy(S.B, S.Bp, sizeof(double) * (size_t)nrows);
                }
                counters->windows_checked++;
                int64_t nf = orc_detect(nrows, S.Bn, S.Bp, eps, S.rflag);
                if (nf == 0) break;
                for (int64_t l = 0; l < nrows; l++)
                    if (S.rflag[l])
                        emit(&S, t0 + k - 1, ORC_EV_WINDOW_FLAG, (int)(l / p->ny),
                             (int)(l % p->ny), attempt, S.Bn[l], S.Bp[l]);
                if (attempt == 0) counters->windows_flagged++;
                if (!auto_correct) {
                    halt = 1;
                    break;
                }
                if (attempt == 1) {
                    counters->persistent++;
                    emit(&S, t0 + k - 1, ORC_EV_PERSISTENT, -1, -1, -1, (double)nf, 0.0);
                    break;
                }
                counters->rollbacks++;
                emit(&S, t0, ORC_EV_ROLLBACK, -1, -1, (int)k, 0.0, 0.0);
                if (S.input_check) verify_checkpoint(&S, t0, ckpt, Bck, Wck);
                memcpy(u_a, ckpt, bytes);
                attempt = 1;
            }
            counters->sweeps_done = t0 + k;
            if (halt) break;
            memcpy(ckpt, u_a, bytes);
            memcpy(Bck, S.Bn, sizeof(double) * (size_t)nrows);
            if (S.input_check) orc_weighted_row_checksums(p, u_a, Wck);
            t0 += k;
        }
        free(ckpt);
        free(Bck);
        free(Wck);
        free(hist);
    }

    free(S.B);
    free(S.Bn);
    free(S.Bp);
    free(S.cB);
    free(S.cA);
    free(S.At);
    free(S.An);
    free(S.Ap);
    free(S.rs);
    free(S.cs);
    free(S.rflag);
    free(S.cflag);
    free(S.W);
    free(S.Wn);
    free(S.Bi);
    free(S.mflag);
    free(S.w);
    return 0;
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
