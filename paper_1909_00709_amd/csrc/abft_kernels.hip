// gfx950 kernels other than the sweep: locate and correct (Section 3.5), the offline window
// check (Section 4.1), and the initial checksums.
#include <algorithm>

#include "abft_device.h"

namespace abft {

constexpr int kFixXPT = 4;  // columns per thread in the locate block: nx <= 4 * kFixBlock

// Deterministic block-wide fp64 sum (fixed combination order).
__device__ double block_sum(double v, double* red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum(v);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w];
    __syncthreads();
    return s;
}

// ------------------------------------------------------------------------------------------
// Repair of input points changed in memory (found by the sweep's input-side check).
// ------------------------------------------------------------------------------------------

// G(u, x, y, z): the grid extended by the boundary rule (constant ghosts outside).
template <typename T>
__device__ __forceinline__ T ghost_value(const FixArgs& a, const T* u, int x, int y, int z)
{
    const int bc = a.st.bc;
    const int mx = map_coord(x, a.nx, bc), my = map_coord(y, a.ny, bc), mz = map_coord(z, a.nz, bc);
    if (mx < 0 || my < 0 || mz < 0) return (T)a.st.g;
    return u[((size_t)mz * a.ny + my) * a.nx + mx];
}

// The locate/correct helpers below take the kernel's by-value arguments by reference and are
// force-inlined: as real calls, the radius-2 and box variants had the arguments (with the
// stencil's weights) copied into private memory, 552-656 bytes per lane, and even their
// fault-free launch, which exits at once, took about twice as long.

// Eq.(1) at one point with the operations of the sweep kernels in their order (the constant
// term, then one fused multiply-add per tap, absent taps adding zero), so that the value is
// the one the sweep stores for the same input.
template <typename T, int RAD, int BOX>
__device__ __forceinline__ T point_value(const FixArgs& a, const T* u, int x, int y, int z)
{
    const size_t i = ((size_t)z * a.ny + y) * a.nx + x;
    T acc = a.C != nullptr ? static_cast<const T*>(a.C)[i] : (T)a.c_scalar;
    if constexpr (BOX) {
        // unrolled: constant tap indices keep the weights out of private memory
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const int sl = box_slot(dx, dy, dz);
                    const bool on = (a.st.bmask >> sl) & 1u;
                    acc = fma((T)a.st.wb[sl], on ? ghost_value(a, u, x + dx, y + dy, z + dz) : T(0),
                              acc);
                }
    } else {
        auto tap = [&](int slot, int dx, int dy, int dz) {
            const bool on = (a.st.mask >> slot) & 1u;
            acc = fma((T)a.st.w[slot], on ? ghost_value(a, u, x + dx, y + dy, z + dz) : T(0), acc);
        };
        tap(W_C, 0, 0, 0);
        for (int d = 1; d <= RAD; ++d) {
            tap(w_slot(0, d, -1), -d, 0, 0);
            tap(w_slot(0, d, 1), d, 0, 0);
            tap(w_slot(1, d, -1), 0, -d, 0);
            tap(w_slot(1, d, 1), 0, d, 0);
            tap(w_slot(2, d, -1), 0, 0, -d);
            tap(w_slot(2, d, 1), 0, 0, d);
        }
    }
    return acc;
}

// x-boundary term of Theorem 1 for a shift dx (|dx| <= 2) of input row (z, y), which may lie
// outside the grid (a row of constant ghosts has none): dx < 0 reads G(dx .. -1) and drops
// u(nx+dx .. nx-1); dx > 0 reads G(nx .. nx+dx-1) and drops u(0 .. dx-1).
template <typename T>
__device__ __forceinline__ double row_boundary_term(const FixArgs& a, const T* u, int z, int y, int dx)
{
    if (map_coord(z, a.nz, a.st.bc) < 0 || map_coord(y, a.ny, a.st.bc) < 0) return 0.0;
    double b = 0.0;
    if (dx < 0)
        for (int q = 1; q <= -dx; ++q)
            b += (double)ghost_value(a, u, -q, y, z) - (double)ghost_value(a, u, a.nx - q, y, z);
    else
        for (int q = 0; q < dx; ++q)
            b += (double)ghost_value(a, u, a.nx + q, y, z) - (double)ghost_value(a, u, q, y, z);
    return b;
}

// Theorem 1's prediction of output row (z, y) from the input's checksums and boundary values,
// as the sweep forms it.
template <typename T, int RAD, int BOX>
__device__ __forceinline__ double predict_row(const FixArgs& a, const T* u, int z, int y)
{
    const int bc = a.st.bc, nx = a.nx;
    auto brow = [&](int z2, int y2) -> double {
        const int mz = map_coord(z2, a.nz, bc), my = map_coord(y2, a.ny, bc);
        if (mz < 0 || my < 0) return (double)nx * a.st.g;
        return a.Bt[(size_t)mz * a.ny + my];
    };
    const size_t l = (size_t)z * a.ny + y;
    double bp = a.cB[l];
    if constexpr (BOX) {
        double e = 0.0;
        // unrolled, as in point_value
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
                const int sm = box_slot(-1, dy, dz), sp = box_slot(1, dy, dz);
                if ((a.st.bmask >> sm) & 1u) e += a.st.wb[sm] * row_boundary_term(a, u, z + dz, y + dy, -1);
                if ((a.st.bmask >> sp) & 1u) e += a.st.wb[sp] * row_boundary_term(a, u, z + dz, y + dy, 1);
            }
        bp += e;
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
                double wsum = 0.0;
                bool any = false;
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const int sl = box_slot(dx, dy, dz);
                    if ((a.st.bmask >> sl) & 1u) {
                        wsum += a.st.wb[sl];
                        any = true;
                    }
                }
                if (any) bp += wsum * brow(z + dz, y + dy);
            }
    } else {
        const uint32_t m = a.st.mask;
        const double b0 = a.Bt[l];
        if (m & (1u << W_C)) bp += a.st.w[W_C] * b0;
        double e = 0.0;
        for (int d = 1; d <= RAD; ++d) {
            if (m & (1u << w_slot(0, d, -1))) {
                bp += a.st.w[w_slot(0, d, -1)] * b0;
                e += a.st.w[w_slot(0, d, -1)] * row_boundary_term(a, u, z, y, -d);
            }
            if (m & (1u << w_slot(0, d, 1))) {
                bp += a.st.w[w_slot(0, d, 1)] * b0;
                e += a.st.w[w_slot(0, d, 1)] * row_boundary_term(a, u, z, y, d);
            }
        }
        bp += e;
        for (int d = 1; d <= RAD; ++d) {
            if (m & (1u << w_slot(1, d, -1))) bp += a.st.w[w_slot(1, d, -1)] * brow(z, y - d);
            if (m & (1u << w_slot(1, d, 1))) bp += a.st.w[w_slot(1, d, 1)] * brow(z, y + d);
            if (m & (1u << w_slot(2, d, -1))) bp += a.st.w[w_slot(2, d, -1)] * brow(z - d, y);
            if (m & (1u << w_slot(2, d, 1))) bp += a.st.w[w_slot(2, d, 1)] * brow(z + d, y);
        }
    }
    return bp;
}

// Output coordinate of the repair window: periodic wraps; the other rules have no outputs
// outside the grid (an output that reads a clamped edge point lies inside the window).
__device__ __forceinline__ int window_coord(int c, int n, int bc)
{
    if (c >= 0 && c < n) return c;
    return bc == ABFT_BC_PERIODIC ? map_coord(c, n, bc) : -1;
}

template <typename T>
__device__ __forceinline__ bool same_bits(T a, T b)
{
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(uint32_t, a) == __builtin_bit_cast(uint32_t, b);
    else
        return __builtin_bit_cast(uint64_t, a) == __builtin_bit_cast(uint64_t, b);
}

// Sum and index-weighted sum of one row, by the whole block (fixed order).
template <typename T>
__device__ void block_row_sums(const T* row, int nx, double* red, double* s, double* w)
{
    double ps = 0.0, pw = 0.0;
    for (int x = threadIdx.x; x < nx; x += kFixBlock) {
        const double v = (double)row[x];
        ps += v;
        pw = fma((double)(x + 1), v, pw);
    }
    *s = block_sum(ps, red);
    *w = block_sum(pw, red);
}

// The sweep's input-side check flagged input rows: the row's sum changed by d = S - B^t, its
// index-weighted sum by (x + 1) d for a single changed point, which places it; the value comes
// back from B^t and the other points of the row (the partial-sum form used for Eq.(10)); the
// outputs of the sweep in the window of the stencil's reach around the point are evaluated
// again, and the checksums of the output rows in the window recomputed.  Returns the number of
// points repaired (the same in every thread).
template <typename T, int RAD, int BOX>
__device__ __forceinline__ int repair_inputs(const FixArgs& a, double* red, int64_t t)
{
    FlagSlot* slot = a.slot;
    const unsigned m_all = slot->mcount;
    if (m_all == 0u || a.Wt == nullptr) return 0;
    const int tid = threadIdx.x;
    if (m_all > (unsigned)kMaxMemFlags) {
        if (tid == 0) {
            atomicAdd(&a.cnt->uncorrectable, 1ull);
            emit_event(a.cnt, a.ev, a.ev_cap, t, ABFT_EV_UNCORRECTABLE, -1, -1, -1,
                       (double)m_all, 1.0, a.grid);
        }
        return 0;
    }
    const int m = (int)m_all;
    if (tid == 0) {  // order by (z, y)
        for (int i = 1; i < m; ++i) {
            const MemFlag key = slot->mrows[i];
            int j = i - 1;
            while (j >= 0 && (slot->mrows[j].z > key.z ||
                              (slot->mrows[j].z == key.z && slot->mrows[j].y > key.y))) {
                slot->mrows[j + 1] = slot->mrows[j];
                --j;
            }
            slot->mrows[j + 1] = key;
        }
    }
    __syncthreads();
    T* uin = static_cast<T*>(const_cast<void*>(a.uin));
    T* uout = static_cast<T*>(a.uout);
    const int nx = a.nx, ny = a.ny, nz = a.nz, bc = a.st.bc;
    constexpr int R = BOX ? 1 : RAD;
    constexpr int NWIN = (2 * R + 1) * (2 * R + 1) * (2 * R + 1);
    static_assert(NWIN <= kFixBlock, "one thread per point of the repair window");
    int nrep = 0;
    for (int i = 0; i < m; ++i) {
        const int z = slot->mrows[i].z, y = slot->mrows[i].y;
        const size_t l = (size_t)z * ny + y;
        T* row = uin + l * nx;
        double S, Wr;
        block_row_sums(row, nx, red, &S, &Wr);
        const double d = S - a.Bt[l];
        const double ratio = (Wr - a.Wt[l]) / d;
        const double pos = rint(ratio);
        if (!isfinite(ratio) || fabs(ratio - pos) > 0.25 || pos < 1.0 || pos > (double)nx) {
            if (tid == 0) {
                atomicAdd(&a.cnt->mem_unlocated, 1ull);
                emit_event(a.cnt, a.ev, a.ev_cap, t, ABFT_EV_MEM_UNLOCATED, z, y, -1, d, ratio,
                           a.grid);
            }
            continue;
        }
        const int x = (int)pos - 1;
        double p = 0.0;
        for (int q = tid; q < nx; q += kFixBlock)
            if (q != x) p += (double)row[q];
        const double rest = block_sum(p, red);
        if (tid == 0) {
            const T old = row[x];
            row[x] = (T)(a.Bt[l] - rest);
            atomicAdd(&a.cnt->mem_corrected, 1ull);
            emit_event(a.cnt, a.ev, a.ev_cap, t, ABFT_EV_MEM_CORRECTED, z, y, x, (double)old,
                       (double)row[x], a.grid);
        }
        __syncthreads();
        if (tid < NWIN) {
            const int ox = tid % (2 * R + 1) - R, oy = (tid / (2 * R + 1)) % (2 * R + 1) - R,
                      oz = tid / ((2 * R + 1) * (2 * R + 1)) - R;
            const int xx = window_coord(x + ox, nx, bc), yy = window_coord(y + oy, ny, bc),
                      zz = window_coord(z + oz, nz, bc);
            if (xx >= 0 && yy >= 0 && zz >= 0)
                uout[((size_t)zz * ny + yy) * nx + xx] = point_value<T, RAD, BOX>(a, uin, xx, yy, zz);
        }
        __syncthreads();
        for (int oz = -R; oz <= R; ++oz)
            for (int oy = -R; oy <= R; ++oy) {
                const int yy = window_coord(y + oy, ny, bc), zz = window_coord(z + oz, nz, bc);
                if (yy < 0 || zz < 0) continue;
                const size_t lo = (size_t)zz * ny + yy;
                double So, Wo;
                block_row_sums(uout + lo * nx, nx, red, &So, &Wo);
                if (tid == 0) {
                    a.Bn[lo] = So;
                    a.Wn[lo] = Wo;
                }
            }
        __syncthreads();
        ++nrep;
    }
    return nrep;
}

// ------------------------------------------------------------------------------------------
// Location and correction on the tiles of one layer (tile-local checksums).  The flagged
// tiles are slot->rows[i .. j) (sorted by y, then tile), the layer's flagged columns xs[0 .. K)
// (ascending).  The candidates of a tile are the flagged columns inside its x range.  A
// flagged tile without one is a checksum-side mismatch.  A candidate alone in its tile takes
// the tile checksum's value (its predicted sum minus the tile's other points), alone in its
// column the column's, alone in both their mean; a candidate shared both ways makes the layer
// uncorrectable.  With the recompute correction every candidate is evaluated again.  Then the
// flagged tiles' sums are recomputed.
// ------------------------------------------------------------------------------------------
template <typename T, int RAD>
__device__ __forceinline__ void fix_tiles_layer(const FixArgs& a, int i, int j, int z, const int* xs, int K,
                                const double* Ap, double* red, int& sh, int64_t t)
{
    FlagSlot* slot = a.slot;
    const int tid = threadIdx.x, TT = a.tile_x, nx = a.nx, ny = a.ny, ntx = nx / TT;
    const size_t ps = (size_t)nx * (size_t)ny;
    T* uout = static_cast<T*>(a.uout);
    const T* uin = static_cast<const T*>(a.uin);
    // first flagged column at or after x (xs ascending)
    auto first_col = [&](int x) {
        int lo = 0, hi = K;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (xs[mid] < x) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    // flagged tiles of the layer with tile index k
    auto tiles_at = [&](int k) {
        int n = 0;
        for (int ri = i; ri < j; ++ri) n += slot->rows[ri].k == k;
        return n;
    };
    if (tid == 0) {
        int ambiguous = 0, nc = 0;
        for (int ri = i; ri < j; ++ri) {
            const RowFlag& rf = slot->rows[ri];
            const int c0 = first_col(rf.k * TT), c1 = first_col(rf.k * TT + TT);
            const int nin = c1 - c0;
            nc += nin;
            if (nin == 0) {
                atomicAdd(&a.cnt->checksum_faults, 1ull);
                emit_event(a.cnt, a.ev, a.ev_cap, t, ABFT_EV_CHECKSUM_FAULT, z, rf.y, rf.k * TT,
                           rf.direct, rf.pred, a.grid);
            } else if (nin > 1 && tiles_at(rf.k) > 1) {
                ambiguous = 1;
            }
        }
        const bool can = a.recompute ? nc <= kMaxRecompute : !ambiguous;
        if (nc > 0 && !can) {
            atomicAdd(&a.cnt->uncorrectable, 1ull);
            emit_event(a.cnt, a.ev, a.ev_cap, t, ABFT_EV_UNCORRECTABLE, z, -1, -1,
                       (double)(j - i), (double)K, a.grid);
        }
        sh = (nc > 0 && can) ? 1 : 0;
    }
    __syncthreads();
    const bool correct = sh != 0;
    __syncthreads();
    if (correct) {
        for (int ri = i; ri < j; ++ri) {
            const RowFlag rf = slot->rows[ri];
            const int c0 = first_col(rf.k * TT), c1 = first_col(rf.k * TT + TT);
            const int nin = c1 - c0;
            T* row = uout + (size_t)z * ps + (size_t)rf.y * nx;
            if (a.recompute) {
                for (int q = c0 + tid; q < c1; q += kFixBlock) {
                    const int x = xs[q];
                    const T old = row[x];
                    const T nv = point_value<T, RAD, 0>(a, uin, x, rf.y, z);
                    if (!same_bits(old, nv)) {
                        row[x] = nv;
                        atomicAdd(&a.cnt->corrected, 1ull);
                        emit_event(a.cnt, a.ev, a.ev_cap, t, ABFT_EV_CORRECTED, z, rf.y, x,
                                   (double)old, (double)nv, a.grid);
                    }
                }
                continue;
            }
            const int ncol = tiles_at(rf.k);  // candidates in each of this tile's columns
            for (int q = c0; q < c1; ++q) {
                const int x = xs[q];
                double vt = 0.0, vc = 0.0;
                if (nin == 1) {
                    double p = 0.0;
                    for (int xx = rf.k * TT + tid; xx < rf.k * TT + TT; xx += kFixBlock)
                        if (xx != x) p += (double)row[xx];
                    vt = rf.pred - block_sum(p, red);
                }
                if (ncol == 1) {
                    double p = 0.0;
                    for (int yy = tid; yy < ny; yy += kFixBlock)
                        if (yy != rf.y) p += (double)uout[(size_t)z * ps + (size_t)yy * nx + x];
                    vc = Ap[x] - block_sum(p, red);
                }
                if (tid == 0) {
                    const double v = (nin == 1 && ncol == 1) ? 0.5 * (vt + vc)
                                                             : (nin == 1 ? vt : vc);
                    const T old = row[x];
                    row[x] = (T)v;
                    atomicAdd(&a.cnt->corrected, 1ull);
                    emit_event(a.cnt, a.ev, a.ev_cap, t, ABFT_EV_CORRECTED, z, rf.y, x,
                               (double)old, (double)(T)v, a.grid);
                }
                __syncthreads();
            }
        }
        __syncthreads();
    }
    // checksum update of the flagged tiles
    for (int ri = i; ri < j; ++ri) {
        const RowFlag rf = slot->rows[ri];
        const T* row = uout + (size_t)z * ps + (size_t)rf.y * nx + (size_t)rf.k * TT;
        double p = 0.0;
        for (int xx = tid; xx < TT; xx += kFixBlock) p += (double)row[xx];
        const double S = block_sum(p, red);
        if (tid == 0) a.Bn[((size_t)z * ny + rf.y) * ntx + rf.k] = S;
    }
}

// ------------------------------------------------------------------------------------------
// Tile-local checksums: Theorem 1 on every tile and the comparison.  A thread owns one tile
// position (y, k) and marches along a slab of planes, keeping the tile sums of the planes
// z-2 .. z+2 in registers, so each input tile sum is read about once; the y-neighbours come
// through the cache.
// ------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) tile_check_kernel(const TileCheckArgs a, int slab)
{
    const int TT = a.tile_x, ntx = a.nx / TT, ny = a.ny, nz = a.nz, bc = a.st.bc;
    const int64_t nyt = (int64_t)ny * ntx;
    const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int zs = (int)blockIdx.y * slab, ze = min(zs + slab, nz);
    const int64_t t = a.t_off + (a.t_base != nullptr ? *a.t_base : 0);
    const unsigned long long known = noise_known(a.cnt);
    double noise = 0.0;
    if (col < nyt) {
        const int k = (int)(col % ntx), y = (int)(col / ntx);
        const uint32_t m = a.st.mask;
        const double ghost_sum = (double)TT * a.st.g;
        auto btile = [&](int z2, int y2) -> double {
            const int mz = map_coord(z2, nz, bc), my = map_coord(y2, ny, bc);
            if (mz < 0 || my < 0) return ghost_sum;
            return a.Bt[((size_t)mz * ny + my) * ntx + k];
        };
        auto has = [&](int slot) { return (m >> slot) & 1u; };
        double win[5];  // tile sums of the planes z-2 .. z+2 at (y, k)
        for (int q = 0; q < 5; ++q) win[q] = btile(zs - 2 + q, y);
        // the loads of plane z+1 are issued before plane z is compared, so that they are in
        // flight while a flag (rare) is recorded
        struct Plane {
            double cb, e, s, ym[2], yp[2];
        };
        auto load_plane = [&](int z, Plane& P) {
            const size_t i = ((size_t)z * ny + y) * ntx + k;
            P.cb = a.cB[i];
            P.e = a.Et[i];
            P.s = a.Bn[i];
            for (int d = 1; d <= 2; ++d) {
                P.ym[d - 1] = has(w_slot(1, d, -1)) ? btile(z, y - d) : 0.0;
                P.yp[d - 1] = has(w_slot(1, d, 1)) ? btile(z, y + d) : 0.0;
            }
        };
        Plane cur, nxt;
        load_plane(zs, cur);
        for (int z = zs; z < ze; ++z) {
            if (z + 1 < ze) load_plane(z + 1, nxt);
            const double win_next = btile(z + 3, y);
            // the order of the terms follows the whole-row prediction of the sweep
            double bp = cur.cb;
            if (has(W_C)) bp += a.st.w[W_C] * win[2];
            for (int d = 1; d <= 2; ++d) {
                if (has(w_slot(0, d, -1))) bp += a.st.w[w_slot(0, d, -1)] * win[2];
                if (has(w_slot(0, d, 1))) bp += a.st.w[w_slot(0, d, 1)] * win[2];
            }
            bp += cur.e;
            for (int d = 1; d <= 2; ++d) {
                if (has(w_slot(1, d, -1))) bp += a.st.w[w_slot(1, d, -1)] * cur.ym[d - 1];
                if (has(w_slot(1, d, 1))) bp += a.st.w[w_slot(1, d, 1)] * cur.yp[d - 1];
                if (has(w_slot(2, d, -1))) bp += a.st.w[w_slot(2, d, -1)] * win[2 - d];
                if (has(w_slot(2, d, 1))) bp += a.st.w[w_slot(2, d, 1)] * win[2 + d];
            }
            const double S = cur.s;
            const double dlt = fabs(S - bp);
            if (!(dlt <= a.eps * fabs(bp))) {
                const unsigned f = atomicAdd(&a.slot->count, 1u);
                if (f < (unsigned)kMaxFlags) {
                    RowFlag rf;
                    rf.z = z;
                    rf.y = y;
                    rf.k = k;
                    rf.pad = 0;
                    rf.direct = S;
                    rf.pred = bp;
                    a.slot->rows[f] = rf;
                } else {
                    atomicAdd(&a.cnt->overflow, 1ull);
                }
                atomicAdd(&a.cnt->rows_flagged, 1ull);
                emit_event(a.cnt, a.ev, a.ev_cap, t, ABFT_EV_ROW_FLAG, z, y, k * TT, S, bp,
                           a.grid);
            } else if (bp != 0.0) {
                noise = fmax(noise, dlt / fabs(bp));
            }
            for (int q = 0; q < 4; ++q) win[q] = win[q + 1];
            win[4] = win_next;
            cur = nxt;
        }
    }
    record_noise(a.cnt, noise, known);
}

// ------------------------------------------------------------------------------------------
// Locate and correct after a sweep whose row checks flagged something (Sections 3.4-3.5).
// One block.  For each layer with flagged rows: the column checksums of the layer (Eq.(2)),
// their prediction from the input grid (Theorem 1, Eq.(4)), the flagged columns, and the
// correction of the intersections (Eq.(10), with the partial sum over the other points taken
// directly).  Exits at once when nothing was flagged.
// ------------------------------------------------------------------------------------------
template <typename T, int RAD, int BOX>
__device__ __forceinline__ void fixup_body(const FixArgs& a, unsigned char* smem_raw, double* red, int& sh_K)
{
    FlagSlot* slot = a.slot;
    if (slot->count == 0u && slot->mcount == 0u) return;  // nothing flagged: the usual case
    const int64_t t0 = a.t_off + (a.t_base != nullptr ? *a.t_base : 0);
    // input points changed in memory first: the output rows they reached are then tested
    // again against predictions from the repaired input, and only rows still mismatched go on
    const int nrep = repair_inputs<T, RAD, BOX>(a, red, t0);
    if (nrep > 0 && slot->count > 0u && slot->count <= (unsigned)kMaxFlags) {
        const int nf = (int)slot->count;
        int* keep = reinterpret_cast<int*>(smem_raw);  // [kMaxFlags]
        for (int i = threadIdx.x; i < nf; i += kFixBlock) {
            RowFlag rf = slot->rows[i];
            rf.direct = a.Bn[(size_t)rf.z * a.ny + rf.y];
            rf.pred = predict_row<T, RAD, BOX>(a, static_cast<const T*>(a.uin), rf.z, rf.y);
            slot->rows[i] = rf;
            keep[i] = !(fabs(rf.direct - rf.pred) <= a.eps * fabs(rf.pred));
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned k = 0;
            for (int i = 0; i < nf; ++i)
                if (keep[i]) slot->rows[k++] = slot->rows[i];
            slot->count = k;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) slot->mcount = 0u;
    const unsigned n_all = slot->count;
    __syncthreads();
    if (n_all == 0u) return;

    const int nx = a.nx, ny = a.ny, nz = a.nz, bc = a.st.bc;
    double* At = reinterpret_cast<double*>(smem_raw);
    double* Ap = At + nx;
    double* An = Ap + nx;
    int* cflag = reinterpret_cast<int*>(An + nx);
    int* xs = cflag + nx;
    // box stencils: column sums and first / last points of the input layers z-1, z, z+1
    double* A3 = reinterpret_cast<double*>(xs + nx);  // [3][nx]
    double* F3 = A3 + 3 * nx;
    double* L3 = F3 + 3 * nx;

    const int tid = threadIdx.x;
    const int64_t t = a.t_off + (a.t_base != nullptr ? *a.t_base : 0);
    const T* uin = static_cast<const T*>(a.uin);
    T* uout = static_cast<T*>(a.uout);
    const size_t ps = (size_t)nx * (size_t)ny;
    const double gd = (double)(T)a.st.g;
    const uint32_t mask = a.st.mask;

    if (n_all > (unsigned)kMaxFlags) {
        // more flagged rows than remembered: nothing can be located reliably
        if (tid == 0) {
            atomicAdd(&a.cnt->uncorrectable, 1ull);
            emit_event(a.cnt, a.ev, a.ev_cap, t, ABFT_EV_UNCORRECTABLE, -1, -1, -1,
                       (double)n_all, 0.0, a.grid);
            slot->count = 0u;
        }
        return;
    }
    const int n = (int)n_all;
    if (tid == 0) {  // order the flagged rows by (z, y)
        for (int i = 1; i < n; ++i) {
            const RowFlag key = slot->rows[i];
            int j = i - 1;
            while (j >= 0 && (slot->rows[j].z > key.z ||
                              (slot->rows[j].z == key.z && (slot->rows[j].y > key.y ||
                                                            (slot->rows[j].y == key.y &&
                                                             slot->rows[j].k > key.k))))) {
                slot->rows[j + 1] = slot->rows[j];
                --j;
            }
            slot->rows[j + 1] = key;
        }
    }
    __syncthreads();

    int i = 0;
    while (i < n) {
        const int z = slot->rows[i].z;
        int j = i;
        while (j < n && slot->rows[j].z == z) ++j;
        const int R = j - i;
        if constexpr (BOX) {
            // column sums and end points of the input layers z-1, z, z+1 (mapped), and the
            // output layer's column sums
            for (int x = tid; x < nx; x += kFixBlock) {
#pragma unroll
                for (int dz = -1; dz <= 1; ++dz) {
                    const int mz = map_coord(z + dz, nz, bc);
                    double sacc = 0.0, f = gd, l = gd;
                    if (mz >= 0) {
                        const T* col = uin + (size_t)mz * ps + x;
                        for (int yy = 0; yy < ny; ++yy) sacc += (double)col[(size_t)yy * nx];
                        f = (double)col[0];
                        l = (double)col[(size_t)(ny - 1) * nx];
                    } else {
                        sacc = (double)ny * gd;
                    }
                    A3[(dz + 1) * nx + x] = sacc;
                    F3[(dz + 1) * nx + x] = f;
                    L3[(dz + 1) * nx + x] = l;
                }
                double sn = 0.0;
                for (int yy = 0; yy < ny; ++yy) sn += (double)uout[(size_t)z * ps + (size_t)yy * nx + x];
                An[x] = sn;
            }
            __syncthreads();
            for (int x = tid; x < nx; x += kFixBlock) {
                double ap = a.cA[(size_t)z * nx + x];
#pragma unroll
                for (int dz = -1; dz <= 1; ++dz) {
                    const bool zin = map_coord(z + dz, nz, bc) >= 0;
#pragma unroll
                    for (int dx = -1; dx <= 1; ++dx) {
                        const int mx = map_coord(x + dx, nx, bc);
                        const bool in = zin && mx >= 0;
                        const double acol = in ? A3[(dz + 1) * nx + mx] : (double)ny * gd;
                        // y-boundary terms of the column: dy = -1 reads G(-1) and drops
                        // u(ny-1), dy = +1 reads G(ny) and drops u(0); a column of constant
                        // ghosts has none
                        double gm = 0.0, gp = 0.0;
                        if (in) {
                            const double f = F3[(dz + 1) * nx + mx], l = L3[(dz + 1) * nx + mx];
                            const double glo = bc == ABFT_BC_CLAMP ? f : (bc == ABFT_BC_PERIODIC ? l : gd);
                            const double ghi = bc == ABFT_BC_CLAMP ? l : (bc == ABFT_BC_PERIODIC ? f : gd);
                            gm = glo - l;
                            gp = ghi - f;
                        }
#pragma unroll
                        for (int dy = -1; dy <= 1; ++dy) {
                            const int sl_ = box_slot(dx, dy, dz);
                            if (!((a.st.bmask >> sl_) & 1u)) continue;
                            const double w = a.st.wb[sl_];
                            ap += w * (acol + (dy < 0 ? gm : (dy > 0 ? gp : 0.0)));
                        }
                    }
                }
                Ap[x] = ap;
                const double dd = fabs(An[x] - ap);
                cflag[x] = !(dd <= a.eps * fabs(ap));
            }
        } else {
            // layers z - d and z + d for d = 1 .. RAD (mapped by the boundary rule)
            int zl[RAD][2];
    #pragma unroll
            for (int d = 0; d < RAD; ++d) {
                zl[d][0] = map_coord(z - d - 1, nz, bc);
                zl[d][1] = map_coord(z + d + 1, nz, bc);
            }

            // column checksums of the layer (input: z and its z-neighbours; output: z), and the
            // first and last RAD points of each input column (the y-boundary terms)
            double s_z[RAD][2][kFixXPT], u_f[RAD][kFixXPT], u_l[RAD][kFixXPT];
    #pragma unroll
            for (int k = 0; k < kFixXPT; ++k) {
                const int x = tid + k * kFixBlock;
    #pragma unroll
                for (int d = 0; d < RAD; ++d) s_z[d][0][k] = s_z[d][1][k] = u_f[d][k] = u_l[d][k] = 0.0;
                if (x < nx) {
                    double sz = 0.0, sn = 0.0, sl[RAD][2];
    #pragma unroll
                    for (int d = 0; d < RAD; ++d) sl[d][0] = sl[d][1] = 0.0;
    #pragma unroll 4
                    for (int yy = 0; yy < ny; ++yy) {
                        const size_t o = (size_t)yy * nx + x;
                        sz += (double)uin[(size_t)z * ps + o];
    #pragma unroll
                        for (int d = 0; d < RAD; ++d)
    #pragma unroll
                            for (int sg = 0; sg < 2; ++sg)
                                if (zl[d][sg] >= 0) sl[d][sg] += (double)uin[(size_t)zl[d][sg] * ps + o];
                        sn += (double)uout[(size_t)z * ps + o];
                    }
                    At[x] = sz;
                    An[x] = sn;
    #pragma unroll
                    for (int d = 0; d < RAD; ++d) {
    #pragma unroll
                        for (int sg = 0; sg < 2; ++sg)
                            s_z[d][sg][k] = zl[d][sg] >= 0 ? sl[d][sg] : (double)ny * gd;
                        const int yf = d < ny ? d : ny - 1, yl = ny - 1 - d >= 0 ? ny - 1 - d : 0;
                        u_f[d][k] = (double)uin[(size_t)z * ps + (size_t)yf * nx + x];
                        u_l[d][k] = (double)uin[(size_t)z * ps + (size_t)yl * nx + x];
                    }
                }
            }
            __syncthreads();
    #pragma unroll
            for (int k = 0; k < kFixXPT; ++k) {
                const int x = tid + k * kFixBlock;
                if (x < nx) {
                    const double a0 = At[x];
                    // G of the column at y = -q and y = ny - 1 + q (q = 1 .. RAD)
                    auto g_lo = [&](int q) -> double {
                        if (bc == ABFT_BC_CLAMP) return u_f[0][k];
                        if (bc == ABFT_BC_PERIODIC) return u_l[q - 1][k];
                        return gd;
                    };
                    auto g_hi = [&](int q) -> double {
                        if (bc == ABFT_BC_CLAMP) return u_l[0][k];
                        if (bc == ABFT_BC_PERIODIC) return u_f[q - 1][k];
                        return gd;
                    };
                    auto acol = [&](int xx) -> double {
                        const int mx = map_coord(xx, nx, bc);
                        return mx < 0 ? (double)ny * gd : At[mx];
                    };
                    double ap = a.cA[(size_t)z * nx + x];
                    if (mask & (1u << W_C)) ap += a.st.w[W_C] * a0;
    #pragma unroll
                    for (int d = 1; d <= RAD; ++d) {
                        if (mask & (1u << w_slot(0, d, -1))) ap += a.st.w[w_slot(0, d, -1)] * acol(x - d);
                        if (mask & (1u << w_slot(0, d, 1))) ap += a.st.w[w_slot(0, d, 1)] * acol(x + d);
                        // shift dy = -d reads G(-d .. -1) and drops the last d points; dy = +d
                        // reads G(ny .. ny+d-1) and drops the first d points
                        if (mask & (1u << w_slot(1, d, -1))) {
                            double b = 0.0;
                            for (int q = 1; q <= d; ++q) b += g_lo(q) - u_l[q - 1][k];
                            ap += a.st.w[w_slot(1, d, -1)] * (a0 + b);
                        }
                        if (mask & (1u << w_slot(1, d, 1))) {
                            double b = 0.0;
                            for (int q = 1; q <= d; ++q) b += g_hi(q) - u_f[q - 1][k];
                            ap += a.st.w[w_slot(1, d, 1)] * (a0 + b);
                        }
                        if (mask & (1u << w_slot(2, d, -1))) ap += a.st.w[w_slot(2, d, -1)] * s_z[d - 1][0][k];
                        if (mask & (1u << w_slot(2, d, 1))) ap += a.st.w[w_slot(2, d, 1)] * s_z[d - 1][1][k];
                    }
                    Ap[x] = ap;
                    const double dd = fabs(An[x] - ap);
                    cflag[x] = !(dd <= a.eps * fabs(ap));
                }
            }
        }
        __syncthreads();
        if (tid == 0) {
            int K = 0;
            for (int x = 0; x < nx; ++x)
                if (cflag[x]) {
                    xs[K++] = x;
                    atomicAdd(&a.cnt->cols_flagged, 1ull);
                    emit_event(a.cnt, a.ev, a.ev_cap, t, ABFT_EV_COL_FLAG, z, -1, x, An[x], Ap[x],
                               a.grid);
                }
            sh_K = K;
        }
        __syncthreads();
        const int K = sh_K;

        if (a.tile_x > 0) {
            fix_tiles_layer<T, RAD>(a, i, j, z, xs, K, Ap, red, sh_K, t);
        } else if (K == 0) {
            // the layer is consistent column-wise: the mismatch sits in a checksum
            if (tid == 0)
                for (int ri = i; ri < j; ++ri) {
                    atomicAdd(&a.cnt->checksum_faults, 1ull);
                    emit_event(a.cnt, a.ev, a.ev_cap, t, ABFT_EV_CHECKSUM_FAULT, z,
                               slot->rows[ri].y, -1, slot->rows[ri].direct, slot->rows[ri].pred,
                               a.grid);
                }
        } else if (a.recompute && (int64_t)R * K <= kMaxRecompute) {
            // stencil locality: every intersection point evaluated again from the sweep's
            // input, with the sweep's operations; a point that was not corrupted gets its own
            // bits back and is not reported
            const T* uin_t = static_cast<const T*>(a.uin);
            for (int q = tid; q < R * K; q += kFixBlock) {
                const int y = slot->rows[i + q / K].y, x = xs[q % K];
                T* pt = uout + (size_t)z * ps + (size_t)y * nx + x;
                const T old = *pt;
                const T nv = point_value<T, RAD, BOX>(a, uin_t, x, y, z);
                if (!same_bits(old, nv)) {
                    *pt = nv;
                    atomicAdd(&a.cnt->corrected, 1ull);
                    emit_event(a.cnt, a.ev, a.ev_cap, t, ABFT_EV_CORRECTED, z, y, x,
                               (double)old, (double)nv, a.grid);
                }
            }
            __syncthreads();
            for (int ri = i; ri < j; ++ri) {
                const int y = slot->rows[ri].y;
                double S, Wr;
                block_row_sums(uout + (size_t)z * ps + (size_t)y * nx, nx, red, &S, &Wr);
                if (tid == 0) {
                    a.Bn[(size_t)z * ny + y] = S;
                    if (a.Wn != nullptr) a.Wn[(size_t)z * ny + y] = Wr;
                }
            }
        } else if (R >= 2 && K >= 2) {
            if (tid == 0) {
                atomicAdd(&a.cnt->uncorrectable, 1ull);
                emit_event(a.cnt, a.ev, a.ev_cap, t, ABFT_EV_UNCORRECTABLE, z, -1, -1, (double)R,
                           (double)K, a.grid);
            }
        } else {
            for (int ri = i; ri < j; ++ri) {
                const int y = slot->rows[ri].y;
                const double bpred = slot->rows[ri].pred;
                for (int kk = 0; kk < K; ++kk) {
                    const int x = xs[kk];
                    T* row = uout + (size_t)z * ps + (size_t)y * nx;
                    double p = 0.0;
                    for (int xx = tid; xx < nx; xx += kFixBlock)
                        if (xx != x) p += (double)row[xx];
                    const double prow = block_sum(p, red);
                    p = 0.0;
                    for (int yy = tid; yy < ny; yy += kFixBlock)
                        if (yy != y) p += (double)uout[(size_t)z * ps + (size_t)yy * nx + x];
                    const double pcol = block_sum(p, red);
                    if (tid == 0) {
                        const double vrow = bpred - prow, vcol = Ap[x] - pcol;
                        double v;
                        if (R == 1 && K == 1) v = 0.5 * (vrow + vcol);
                        else if (R == 1) v = vcol;  // several points in one row: one per column
                        else v = vrow;              // several points in one column: one per row
                        const T old = row[x];
                        row[x] = (T)v;
                        atomicAdd(&a.cnt->corrected, 1ull);
                        emit_event(a.cnt, a.ev, a.ev_cap, t, ABFT_EV_CORRECTED, z, y, x,
                                   (double)old, (double)(T)v, a.grid);
                    }
                    __syncthreads();
                }
                // checksum update after the correction: the row's direct sum (and its
                // index-weighted sum when the input-side check is on)
                const T* rowc = uout + (size_t)z * ps + (size_t)y * nx;
                double S, Wr;
                block_row_sums(rowc, nx, red, &S, &Wr);
                if (tid == 0) {
                    a.Bn[(size_t)z * ny + y] = S;
                    if (a.Wn != nullptr) a.Wn[(size_t)z * ny + y] = Wr;
                }
            }
        }
        __syncthreads();
        i = j;
    }
    if (tid == 0) slot->count = 0u;
}

template <typename T, int RAD, int BOX>
__global__ void __launch_bounds__(kFixBlock) fixup_kernel(const FixArgs a)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    __shared__ double red[kFixBlock / 64];
    __shared__ int sh_K;
    fixup_body<T, RAD, BOX>(a, smem_raw, red, sh_K);
}

// One block per grid of a batch; each exits at once unless its grid flagged a row.
template <typename T, int RAD, int BOX>
__global__ void __launch_bounds__(kFixBlock) fixup_batch_kernel(const BatchArgs b)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    __shared__ double red[kFixBlock / 64];
    __shared__ int sh_K;
    const int g = blockIdx.x;
    const GridDesc& d = b.grids[g];
    const int p = b.parity;
    if (d.slot[p]->count == 0u && d.slot[p]->mcount == 0u) return;
    FixArgs a{};
    a.uin = d.u[p];
    a.uout = d.u[p ^ 1];
    a.Bn = d.B[p ^ 1];
    a.cA = d.cA;
    a.st = d.st;
    a.nx = d.nx;
    a.ny = d.ny;
    a.nz = d.nz;
    a.eps = b.eps;
    a.slot = d.slot[p];
    a.cnt = b.cnt;
    a.ev = b.ev;
    a.ev_cap = b.ev_cap;
    a.grid = g;
    a.t_base = b.t_base;
    a.t_off = b.t_off;
    a.C = d.C;
    a.c_scalar = d.c_scalar;
    a.recompute = b.recompute;
    a.Bt = d.B[p];
    a.Wt = d.W[p];
    a.Wn = d.W[p ^ 1];
    a.cB = d.cB;
    fixup_body<T, RAD, BOX>(a, smem_raw, red, sh_K);
}

// ------------------------------------------------------------------------------------------
// Offline window check (Section 4.1): the checksum interpolation applied k times from the
// checkpoint's checksums, then compared with the direct checksums at the window end.  Each
// block owns a tile of the (z, y) checksum plane and iterates the plane stencil in LDS on the
// tile plus a halo of ns rows / layers (the ns-step dependency cone), so one launch does ns
// steps: all k of a window up to kCheckChunk, else the window's steps in chunks, each but the
// last writing its tiles' interiors to an intermediate plane.
// ------------------------------------------------------------------------------------------
// Neighbours of a checksum-plane cell under the collapsed stencil: (dy, dz) offsets of the
// k-th neighbour, for a star of radius RAD (4 * RAD neighbours) or a box (8).
__device__ constexpr int nb_count(int rad, int box) { return box ? 8 : 4 * rad; }
__device__ constexpr int nb_dy(int k, int box)
{
    return box ? ((k < 4 ? k : k + 1) % 3) - 1 : ((k & 3) == 0 ? -(k / 4 + 1) : (k & 3) == 1 ? k / 4 + 1 : 0);
}
__device__ constexpr int nb_dz(int k, int box)
{
    return box ? ((k < 4 ? k : k + 1) / 3) - 1 : ((k & 3) == 2 ? -(k / 4 + 1) : (k & 3) == 3 ? k / 4 + 1 : 0);
}

template <int RAD, int BOX>
__global__ void __launch_bounds__(kCheckBlock) check_kernel(const CheckArgs a)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    if (a.guard != nullptr && *a.guard == 0u) return;
    constexpr int NN = nb_count(RAD, BOX);

    const int nx = a.nx, ny = a.ny, nz = a.nz, bc = a.st.bc, k = a.ns, hal = RAD * a.ns;
    const bool per = bc == ABFT_BC_PERIODIC;
    const double gd = a.st.g;
    const uint32_t mask = a.st.mask;
    const int tid = threadIdx.x;
    const int yt = blockIdx.x % a.nyt, zt = blockIdx.x / a.nyt;
    const int iy0 = yt * a.tyi, iy1 = min(iy0 + a.tyi, ny);
    const int iz0 = zt * a.tzi, iz1 = min(iz0 + a.tzi, nz);
    int ry0, ry1, rz0, rz1;
    if (per) {
        ry0 = iy0 - hal; ry1 = iy1 + hal; rz0 = iz0 - hal; rz1 = iz1 + hal;
    } else {
        ry0 = max(0, iy0 - hal); ry1 = min(ny, iy1 + hal);
        rz0 = max(0, iz0 - hal); rz1 = min(nz, iz1 + hal);
    }
    const int RY = ry1 - ry0, RZ = rz1 - rz0, NC = RY * RZ;
    double* cur = reinterpret_cast<double*>(smem_raw);
    double* nxt = cur + (size_t)a.ry_max * a.rz_max;

    auto wrap = [](int c, int n) { const int m = c % n; return m < 0 ? m + n : m; };
    auto wt = [&](int slot) { return ((mask >> slot) & 1u) ? a.st.w[slot] : 0.0; };
    auto wbox = [&](int dy, int dz) {  // the box weights of a (dy, dz) row, summed over dx
        double s = 0.0;
        for (int dx = -1; dx <= 1; ++dx) {
            const int sl = box_slot(dx, dy, dz);
            if ((a.st.bmask >> sl) & 1u) s += a.st.wb[sl];
        }
        return s;
    };
    // the x taps collapse onto the row itself (their boundary terms come from E)
    double wx, wn[NN];
    if constexpr (BOX) {
        wx = wbox(0, 0);
#pragma unroll
        for (int n = 0; n < NN; ++n) wn[n] = wbox(nb_dy(n, 1), nb_dz(n, 1));
    } else {
        wx = wt(W_C);
#pragma unroll
        for (int d = 0; d < RAD; ++d) {
            wx += wt(w_slot(0, d + 1, -1)) + wt(w_slot(0, d + 1, 1));
            wn[4 * d + 0] = wt(w_slot(1, d + 1, -1));
            wn[4 * d + 1] = wt(w_slot(1, d + 1, 1));
            wn[4 * d + 2] = wt(w_slot(2, d + 1, -1));
            wn[4 * d + 3] = wt(w_slot(2, d + 1, 1));
        }
    }

    // Each thread owns the same cells at every step: their constant-term checksums, global
    // offsets and neighbour cells stay in registers.  nb < 0 marks a neighbour that is a row
    // of constant ghosts (sum nx * g); a neighbour outside the loaded region points at the
    // cell itself (its value only reaches cells outside the tile).
    double cbv[kCheckCells];
    int gl[kCheckCells], nb[kCheckCells][NN];
#pragma unroll
    for (int q = 0; q < kCheckCells; ++q) {
        const int i = tid + q * kCheckBlock;
        cbv[q] = 0.0;
        gl[q] = 0;
#pragma unroll
        for (int n = 0; n < NN; ++n) nb[q][n] = i < NC ? i : 0;
        if (i < NC) {
            const int yy = ry0 + i % RY, zz = rz0 + i / RY;
            const int gy = per ? wrap(yy, ny) : yy, gz = per ? wrap(zz, nz) : zz;
            gl[q] = gz * ny + gy;
            cbv[q] = a.cB[gl[q]];
            cur[i] = a.Bin[gl[q]];
            auto nbi = [&](int dz, int dy) -> int {
                int y2 = yy + dy, z2 = zz + dz;
                if (!per && (y2 < 0 || y2 >= ny || z2 < 0 || z2 >= nz)) {
                    if (bc == ABFT_BC_CONSTANT) return -1;
                    y2 = min(max(y2, 0), ny - 1);
                    z2 = min(max(z2, 0), nz - 1);
                }
                if (y2 < ry0 || y2 >= ry1 || z2 < rz0 || z2 >= rz1) return i;
                return (z2 - rz0) * RY + (y2 - ry0);
            };
#pragma unroll
            for (int n = 0; n < NN; ++n) nb[q][n] = nbi(nb_dz(n, BOX), nb_dy(n, BOX));
        }
    }
    __syncthreads();

    const double ghost_row = (double)nx * gd;
    for (int s = 0; s < k; ++s) {
        const double* Es = a.E != nullptr ? a.E + (size_t)(a.s0 + s) * nz * ny : nullptr;
#pragma unroll
        for (int q = 0; q < kCheckCells; ++q) {
            const int i = tid + q * kCheckBlock;
            if (i < NC) {
                auto val = [&](int j) { return j < 0 ? ghost_row : cur[j]; };
                double v = cbv[q] + wx * cur[i];
                if (Es != nullptr) v += Es[gl[q]];
#pragma unroll
                for (int n = 0; n < NN; ++n) v += wn[n] * val(nb[q][n]);
                nxt[i] = v;
            }
        }
        __syncthreads();
        double* tmp = cur;
        cur = nxt;
        nxt = tmp;
    }

    if (a.Bout != nullptr) {  // an intermediate chunk: hand the tile's interior on
#pragma unroll
        for (int q = 0; q < kCheckCells; ++q) {
            const int i = tid + q * kCheckBlock;
            if (i >= NC) continue;
            const int yy = ry0 + i % RY, zz = rz0 + i / RY;
            if (yy < iy0 || yy >= iy1 || zz < iz0 || zz >= iz1) continue;
            a.Bout[(size_t)zz * ny + yy] = cur[i];
        }
        return;
    }

    double noise = 0.0;
#pragma unroll
    for (int q = 0; q < kCheckCells; ++q) {
        const int i = tid + q * kCheckBlock;
        if (i >= NC) continue;
        const int yy = ry0 + i % RY, zz = rz0 + i / RY;
        if (yy < iy0 || yy >= iy1 || zz < iz0 || zz >= iz1) continue;
        const double bp = cur[i];
        const double S = a.Bdir[(size_t)zz * ny + yy];
        const double d = fabs(S - bp);
        if (!(d <= a.eps * fabs(bp))) {
            atomicAdd(a.flag_count, 1u);
            emit_event(a.cnt, a.ev, a.ev_cap, a.t_last, ABFT_EV_WINDOW_FLAG, zz, yy, a.attempt, S,
                       bp, 0);
        } else if (bp != 0.0) {
            noise = fmax(noise, d / fabs(bp));
        }
    }
    record_noise(a.cnt, noise);
    __syncthreads();
    if (tid == 0) {
        if (blockIdx.x == 0) atomicAdd(&a.cnt->windows_checked, 1ull);
        __threadfence();
        const unsigned tk = atomicAdd(a.ticket, 1u);
        if (tk == gridDim.x - 1) {  // last block of the check
            atomicExch(a.ticket, 0u);
            const unsigned total = atomicAdd(a.flag_count, 0u);
            if (total > 0u) {
                if (a.attempt == 0) {
                    atomicAdd(&a.cnt->windows_flagged, 1ull);
                } else {
                    atomicAdd(&a.cnt->persistent, 1ull);
                    emit_event(a.cnt, a.ev, a.ev_cap, a.t_last, ABFT_EV_PERSISTENT, -1, -1, -1,
                               (double)total, 0.0, 0);
                }
            }
        }
    }
}

// First sweep of a rollback recompute: records the rollback (guarded like the recompute).
__global__ void rollback_note_kernel(const uint32_t* guard, Counters* cnt, abft_event* ev,
                                     int cap, int64_t t_first, int k)
{
    if (guard != nullptr && *guard == 0u) return;
    if (threadIdx.x == 0) {
        atomicAdd(&cnt->rollbacks, 1ull);
        emit_event(cnt, ev, cap, t_first, ABFT_EV_ROLLBACK, -1, -1, k, 0.0, 0.0, 0);
    }
}

// ------------------------------------------------------------------------------------------
// Initial checksums: row sums (one wavefront per row) and column sums (one thread per column).
// ------------------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) row_sums_kernel(const T* u, double cs, int nx,
                                                        int64_t nrows, double* out)
{
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= nrows) return;
    double p = 0.0;
    for (int x = lane; x < nx; x += 64) p += u != nullptr ? (double)u[row * nx + x] : cs;
    const double s = wave_sum(p);
    if (lane == 0) out[row] = s;
}

template <typename T>
__global__ void __launch_bounds__(256) weighted_row_sums_kernel(const T* u, int nx,
                                                                 int64_t nrows, double* out)
{
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= nrows) return;
    double p = 0.0;
    for (int x = lane; x < nx; x += 64) p = fma((double)(x + 1), (double)u[row * nx + x], p);
    const double s = wave_sum(p);
    if (lane == 0) out[row] = s;
}

// Memory-resident faults of the plan for one sweep: XOR the bit into the sweep's input grid
// before the sweep reads it (kind MEMORY, first attempt, grid 0).  One wavefront walks the
// sweep's entries.
template <typename T>
__global__ void __launch_bounds__(64) mem_flip_kernel(T* u, int nx, int ny,
                                                       const abft_fault* faults,
                                                       const int32_t* first, int64_t tmax,
                                                       const int64_t* t_base, int64_t t_off)
{
    const int64_t t = t_off + (t_base != nullptr ? *t_base : 0);
    if (t < 0 || t >= tmax) return;
    for (int f = first[t] + (int)threadIdx.x; f < first[t + 1]; f += 64) {
        const abft_fault F = faults[f];
        if (F.kind != ABFT_FAULT_MEMORY || F.attempt != 0 || F.grid != 0) continue;
        T* p = u + ((size_t)F.z * ny + F.y) * nx + F.x;
        if constexpr (sizeof(T) == 4)
            *p = __builtin_bit_cast(T, __builtin_bit_cast(uint32_t, *p) ^ (1u << F.bit));
        else
            *p = __builtin_bit_cast(T, __builtin_bit_cast(uint64_t, *p) ^ (1ull << F.bit));
    }
}

// Offline, before a rollback (only when the window check flagged, *guard != 0): the
// checkpoint's rows against the checksums stored when it was formed.  A mismatched row's
// single changed point is placed with the weighted sums kept with the checkpoint and restored
// from the row checksum and the row's other points, so that the recompute starts from the
// checkpoint as it was written.  One wavefront per row; a fixed grid of blocks walks the rows,
// so that an unflagged window costs one short launch.
template <typename T>
__global__ void __launch_bounds__(256) verify_ckpt_kernel(T* u, const double* Bck,
                                                           const double* Wck, int nx, int ny,
                                                           int64_t nrows, double eps,
                                                           const uint32_t* guard, Counters* cnt,
                                                           abft_event* ev, int cap,
                                                           int64_t t_first)
{
    if (guard != nullptr && *guard == 0u) return;
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); row < nrows; row += nw) {
        T* r = u + row * nx;
        double ps = 0.0, pw = 0.0;
        for (int x = lane; x < nx; x += 64) {
            const double v = (double)r[x];
            ps += v;
            pw = fma((double)(x + 1), v, pw);
        }
        const double S = wave_sum(ps), Wr = wave_sum(pw);
        const double B = Bck[row];
        if (fabs(S - B) <= eps * fabs(B)) continue;  // the row is as it was written
        const int z = (int)(row / ny), y = (int)(row % ny);
        if (lane == 0) {
            atomicAdd(&cnt->mem_flagged, 1ull);
            emit_event(cnt, ev, cap, t_first, ABFT_EV_MEM_FLAG, z, y, -1, S, B, 0);
        }
        const double d = S - B;
        const double ratio = (Wr - Wck[row]) / d;
        const double pos = rint(ratio);
        if (!isfinite(ratio) || fabs(ratio - pos) > 0.25 || pos < 1.0 || pos > (double)nx) {
            if (lane == 0) {
                atomicAdd(&cnt->mem_unlocated, 1ull);
                emit_event(cnt, ev, cap, t_first, ABFT_EV_MEM_UNLOCATED, z, y, -1, d, ratio, 0);
            }
            continue;
        }
        const int xp = (int)pos - 1;
        double pr = 0.0;
        for (int x = lane; x < nx; x += 64)
            if (x != xp) pr += (double)r[x];
        const double rest = wave_sum(pr);
        if (lane == 0) {
            const T old = r[xp];
            r[xp] = (T)(B - rest);
            atomicAdd(&cnt->mem_corrected, 1ull);
            emit_event(cnt, ev, cap, t_first, ABFT_EV_MEM_CORRECTED, z, y, xp, (double)old,
                       (double)r[xp], 0);
        }
    }
}

// The same for a batch: each entry flips the input buffer of its own grid.
template <typename T>
__global__ void __launch_bounds__(64) mem_flip_batch_kernel(const GridDesc* grids, int parity,
                                                             const abft_fault* faults,
                                                             const int32_t* first, int64_t tmax,
                                                             const int64_t* t_base,
                                                             int64_t t_off)
{
    const int64_t t = t_off + (t_base != nullptr ? *t_base : 0);
    if (t < 0 || t >= tmax) return;
    for (int f = first[t] + (int)threadIdx.x; f < first[t + 1]; f += 64) {
        const abft_fault F = faults[f];
        if (F.kind != ABFT_FAULT_MEMORY || F.attempt != 0) continue;
        const GridDesc& d = grids[F.grid];
        T* p = static_cast<T*>(d.u[parity]) + ((size_t)F.z * d.ny + F.y) * d.nx + F.x;
        if constexpr (sizeof(T) == 4)
            *p = __builtin_bit_cast(T, __builtin_bit_cast(uint32_t, *p) ^ (1u << F.bit));
        else
            *p = __builtin_bit_cast(T, __builtin_bit_cast(uint64_t, *p) ^ (1ull << F.bit));
    }
}

template <typename T>
__global__ void __launch_bounds__(256) col_sums_kernel(const T* u, double cs, int nx, int ny,
                                                        int nz, double* out)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)nz * nx) return;
    const int64_t z = idx / nx, x = idx % nx;
    double s = 0.0;
    for (int y = 0; y < ny; ++y)
        s += u != nullptr ? (double)u[(z * ny + y) * nx + x] : cs;
    out[idx] = s;
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void set_i64_kernel(int64_t* p, int64_t v)
{
    if (threadIdx.x == 0) *p = v;
}

// ------------------------------------------------------------------------------------------
// Launchers.
// ------------------------------------------------------------------------------------------
bool sweep_shape_supported(int dtype, const SweepShape& s)
{
    const int vf = dtype == ABFT_F32 ? 4 : 2;
    if (s.tz < 1 || (s.nw != 4 && s.nw != 8) || (s.rad != 1 && s.rad != 2)) return false;
    if (s.box && (s.rad != 1 || s.pf != 1)) return false;
    if (s.nw == 8 && s.nch * s.vec * (vf == 4 ? 4 : 8) > kWideBlockLaneBytes)
        return false;
    if (s.pf == 2)
        return s.rad == 1 && s.vec == vf && s.lpr == 64 && (s.nch == 2 || s.nch == 4);
    if (s.pf != 1) return false;
    if (s.vec == vf) {
        if (s.lpr == 16) return s.nch == 1 || s.nch == 2 || s.nch == 4;
        if (s.lpr == 64) return s.nch == 1 || s.nch == 2 || s.nch == 4 || s.nch == 8;
        return false;
    }
    if (s.vec == 1) return s.lpr == 64 && (s.nch == 4 || s.nch == 16);
    return false;
}

int sweep_rows_per_block(const SweepShape& s) { return s.nw * (64 / s.lpr); }

size_t sweep_lds_bytes(int dtype, int nx, const SweepShape& s, bool input_check)
{
    const size_t es = dtype == ABFT_F32 ? 4 : 8;
    const size_t ty = (size_t)sweep_rows_per_block(s);
    const size_t pad = (size_t)std::max(s.vec, s.rad);
    const size_t planes = 2;  // two alternating plane buffers
    // checksum, boundary term[, input, weighted], partial prediction
    const size_t tables = input_check ? 5 : 3;
    return planes * (ty + 2 * s.rad) * (nx + 2 * pad) * es  // plane buffers with halo rows
           + tables * ty * (size_t)s.tz * sizeof(double);
}

hipError_t launch_sweep(int dtype, int mode, int csum, const SweepShape& s, const SweepArgs& a,
                        hipStream_t st)
{
    if (!sweep_shape_supported(dtype, s)) return hipErrorInvalidValue;
    const size_t lds = sweep_lds_bytes(dtype, a.nx, s,
                                       mode == MODE_PROTM || (mode == MODE_CSUM && a.Wn));
    if (mode == MODE_PLAIN) csum = CS_F64;  // no checksum in the plain variant
    if (mode == MODE_TILE) {
        if (s.box || s.vec != 16 / (dtype == ABFT_F32 ? 4 : 8) || a.Bn == nullptr ||
            a.Et == nullptr)
            return hipErrorInvalidValue;
        return dtype == ABFT_F32 ? launch_sweep_f32_tile(csum, s, a, st, lds)
                                 : launch_sweep_f64_tile(csum, s, a, st, lds);
    }
    if (mode == MODE_PROTM) {
        if (a.Wn == nullptr) return hipErrorInvalidValue;
        const bool f32 = dtype == ABFT_F32;
        if (s.box)
            return f32 ? launch_sweep_box_f32_protm(csum, s, a, st, lds)
                       : launch_sweep_box_f64_protm(csum, s, a, st, lds);
        if (s.rad == 2)
            return f32 ? launch_sweep_r2_f32_protm(csum, s, a, st, lds)
                       : launch_sweep_r2_f64_protm(csum, s, a, st, lds);
        return f32 ? launch_sweep_f32_protm(csum, s, a, st, lds)
                   : launch_sweep_f64_protm(csum, s, a, st, lds);
    }
    if (s.box) {
        if (dtype == ABFT_F32) return launch_sweep_box_f32(mode, csum, s, a, st, lds);
        return launch_sweep_box_f64(mode, csum, s, a, st, lds);
    }
    if (s.rad == 2) {
        if (dtype == ABFT_F32) {
            if (mode == MODE_PROT) return launch_sweep_r2_f32_prot(csum, s, a, st, lds);
            return launch_sweep_r2_f32_pc(mode, csum, s, a, st, lds);
        }
        return launch_sweep_r2_f64(mode, csum, s, a, st, lds);
    }
    if (dtype == ABFT_F32) {
        if (mode == MODE_PLAIN) return launch_sweep_f32_plain(csum, s, a, st, lds);
        if (mode == MODE_CSUM) return launch_sweep_f32_csum(csum, s, a, st, lds);
        return launch_sweep_f32_prot(csum, s, a, st, lds);
    }
    if (mode == MODE_PLAIN) return launch_sweep_f64_plain(csum, s, a, st, lds);
    if (mode == MODE_CSUM) return launch_sweep_f64_csum(csum, s, a, st, lds);
    return launch_sweep_f64_prot(csum, s, a, st, lds);
}

// The recompute kernel keeps a few bytes of static LDS (its barrier flag) next to the sweep's
// dynamic LDS; shapes are those of the sweep at prefetch depth 1.
bool recover_shape_supported(int dtype, const SweepShape& s)
{
    SweepShape t = s;
    t.pf = 1;
    return sweep_shape_supported(dtype, t);
}

hipError_t launch_recover(int dtype, int csum, const SweepShape& s, const RecoverArgs& r,
                          int num_cus, hipStream_t st)
{
    if (!recover_shape_supported(dtype, s) || r.k < 1 || r.k > kMaxPeriod || num_cus < 1)
        return hipErrorInvalidValue;
    const size_t lds = sweep_lds_bytes(dtype, r.a.nx, s, r.a.Wn != nullptr);
    if (s.box) {
        if (dtype == ABFT_F32) return launch_recover_box_f32(csum, s, r, lds, num_cus, st);
        return launch_recover_box_f64(csum, s, r, lds, num_cus, st);
    }
    if (s.rad == 2) {
        if (dtype == ABFT_F32) return launch_recover_r2_f32(csum, s, r, lds, num_cus, st);
        return launch_recover_r2_f64(csum, s, r, lds, num_cus, st);
    }
    if (dtype == ABFT_F32) return launch_recover_f32(csum, s, r, lds, num_cus, st);
    return launch_recover_f64(csum, s, r, lds, num_cus, st);
}

size_t fixup_lds_bytes(int nx, bool box)
{
    // the column tables of the layer, or the keep flags of the re-test after an input repair
    return std::max((size_t)nx * ((box ? 12 : 3) * sizeof(double) + 2 * sizeof(int)),
                    (size_t)kMaxFlags * sizeof(int));
}

hipError_t launch_fixup_batch(int dtype, const BatchArgs& b, int maxnx, int rad, int box,
                              hipStream_t st)
{
    const size_t lds = fixup_lds_bytes(maxnx, box != 0);
    auto go = [&](auto kern) -> hipError_t {
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(kern, dim3(b.ngrids), dim3(kFixBlock), lds, st, b);
        return hipGetLastError();
    };
    if (dtype == ABFT_F32) {
        if (box) return go(fixup_batch_kernel<float, 1, 1>);
        if (rad == 2) return go(fixup_batch_kernel<float, 2, 0>);
        return go(fixup_batch_kernel<float, 1, 0>);
    }
    if (box) return go(fixup_batch_kernel<double, 1, 1>);
    if (rad == 2) return go(fixup_batch_kernel<double, 2, 0>);
    return go(fixup_batch_kernel<double, 1, 0>);
}

hipError_t launch_fixup(int dtype, const FixArgs& a, hipStream_t st)
{
    const bool box = a.st.box != 0;
    const size_t lds = fixup_lds_bytes(a.nx, box);
    const bool r2 = a.st.rad == 2;
    auto go = [&](auto kern) -> hipError_t {
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(kern, dim3(1), dim3(kFixBlock), lds, st, a);
        return hipGetLastError();
    };
    if (dtype == ABFT_F32) {
        if (box) return go(fixup_kernel<float, 1, 1>);
        if (r2) return go(fixup_kernel<float, 2, 0>);
        return go(fixup_kernel<float, 1, 0>);
    }
    if (box) return go(fixup_kernel<double, 1, 1>);
    if (r2) return go(fixup_kernel<double, 2, 0>);
    return go(fixup_kernel<double, 1, 0>);
}

hipError_t launch_tile_check(const TileCheckArgs& a, hipStream_t st)
{
    if (a.tile_x < 1 || a.nx % a.tile_x) return hipErrorInvalidValue;
    const int64_t nyt = (int64_t)a.ny * (a.nx / a.tile_x);
    const int64_t bx = (nyt + 255) / 256;
    // slabs of planes so that the launch holds about 1024 blocks
    const int nslab = (int)std::min<int64_t>(a.nz, std::max<int64_t>(1, (1024 + bx - 1) / bx));
    const int slab = (a.nz + nslab - 1) / nslab;
    const int nby = (a.nz + slab - 1) / slab;
    hipLaunchKernelGGL(tile_check_kernel, dim3((unsigned)bx, (unsigned)nby), dim3(256), 0, st, a,
                       slab);
    return hipGetLastError();
}

size_t check_lds_bytes(int ry, int rz) { return (size_t)2 * ry * rz * sizeof(double); }

hipError_t launch_check(const CheckArgs& a, hipStream_t st)
{
    const size_t lds = check_lds_bytes(a.ry_max, a.rz_max);
    if (a.st.box)
        hipLaunchKernelGGL((check_kernel<1, 1>), dim3(a.nyt * a.nzt), dim3(kCheckBlock), lds, st, a);
    else if (a.st.rad == 2)
        hipLaunchKernelGGL((check_kernel<2, 0>), dim3(a.nyt * a.nzt), dim3(kCheckBlock), lds, st, a);
    else
        hipLaunchKernelGGL((check_kernel<1, 0>), dim3(a.nyt * a.nzt), dim3(kCheckBlock), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_rollback_note(const uint32_t* guard, Counters* cnt, abft_event* ev, int cap,
                                int64_t t_first, int k, hipStream_t st)
{
    hipLaunchKernelGGL(rollback_note_kernel, dim3(1), dim3(64), 0, st, guard, cnt, ev, cap,
                       t_first, k);
    return hipGetLastError();
}

hipError_t launch_row_sums(int dtype, const void* u, double cs, int nx, int64_t nrows,
                           double* out, hipStream_t st)
{
    const dim3 grid((unsigned)((nrows + 3) / 4));
    if (dtype == ABFT_F32)
        hipLaunchKernelGGL(row_sums_kernel<float>, grid, dim3(256), 0, st,
                           static_cast<const float*>(u), cs, nx, nrows, out);
    else
        hipLaunchKernelGGL(row_sums_kernel<double>, grid, dim3(256), 0, st,
                           static_cast<const double*>(u), cs, nx, nrows, out);
    return hipGetLastError();
}

hipError_t launch_weighted_row_sums(int dtype, const void* u, int nx, int64_t nrows, double* out,
                                    hipStream_t st)
{
    const dim3 grid((unsigned)((nrows + 3) / 4));
    if (dtype == ABFT_F32)
        hipLaunchKernelGGL(weighted_row_sums_kernel<float>, grid, dim3(256), 0, st,
                           static_cast<const float*>(u), nx, nrows, out);
    else
        hipLaunchKernelGGL(weighted_row_sums_kernel<double>, grid, dim3(256), 0, st,
                           static_cast<const double*>(u), nx, nrows, out);
    return hipGetLastError();
}

hipError_t launch_mem_flip(int dtype, void* u, int nx, int ny, const abft_fault* faults,
                           const int32_t* fault_first, int64_t fault_tmax, const int64_t* t_base,
                           int64_t t_off, hipStream_t st)
{
    if (faults == nullptr || fault_first == nullptr || fault_tmax <= 0) return hipSuccess;
    if (dtype == ABFT_F32)
        hipLaunchKernelGGL(mem_flip_kernel<float>, dim3(1), dim3(64), 0, st,
                           static_cast<float*>(u), nx, ny, faults, fault_first, fault_tmax,
                           t_base, t_off);
    else
        hipLaunchKernelGGL(mem_flip_kernel<double>, dim3(1), dim3(64), 0, st,
                           static_cast<double*>(u), nx, ny, faults, fault_first, fault_tmax,
                           t_base, t_off);
    return hipGetLastError();
}

hipError_t launch_verify_ckpt(int dtype, void* u, const double* Bck, const double* Wck, int nx,
                              int ny, int nz, double eps, const uint32_t* guard, Counters* cnt,
                              abft_event* ev, int cap, int64_t t_first, hipStream_t st)
{
    const int64_t nrows = (int64_t)ny * nz;
    const unsigned nb = (unsigned)std::min<int64_t>((nrows + 3) / 4, 1024);
    if (dtype == ABFT_F32)
        hipLaunchKernelGGL(verify_ckpt_kernel<float>, dim3(nb), dim3(256), 0, st,
                           static_cast<float*>(u), Bck, Wck, nx, ny, nrows, eps, guard, cnt, ev,
                           cap, t_first);
    else
        hipLaunchKernelGGL(verify_ckpt_kernel<double>, dim3(nb), dim3(256), 0, st,
                           static_cast<double*>(u), Bck, Wck, nx, ny, nrows, eps, guard, cnt, ev,
                           cap, t_first);
    return hipGetLastError();
}

hipError_t launch_mem_flip_batch(int dtype, const GridDesc* grids, int parity,
                                 const abft_fault* faults, const int32_t* fault_first,
                                 int64_t fault_tmax, const int64_t* t_base, int64_t t_off,
                                 hipStream_t st)
{
    if (faults == nullptr || fault_first == nullptr || fault_tmax <= 0) return hipSuccess;
    if (dtype == ABFT_F32)
        hipLaunchKernelGGL(mem_flip_batch_kernel<float>, dim3(1), dim3(64), 0, st, grids, parity,
                           faults, fault_first, fault_tmax, t_base, t_off);
    else
        hipLaunchKernelGGL(mem_flip_batch_kernel<double>, dim3(1), dim3(64), 0, st, grids,
                           parity, faults, fault_first, fault_tmax, t_base, t_off);
    return hipGetLastError();
}

hipError_t launch_col_sums(int dtype, const void* u, double cs, int nx, int ny, int nz,
                           double* out, hipStream_t st)
{
    const dim3 grid((unsigned)(((int64_t)nz * nx + 255) / 256));
    if (dtype == ABFT_F32)
        hipLaunchKernelGGL(col_sums_kernel<float>, grid, dim3(256), 0, st,
                           static_cast<const float*>(u), cs, nx, ny, nz, out);
    else
        hipLaunchKernelGGL(col_sums_kernel<double>, grid, dim3(256), 0, st,
                           static_cast<const double*>(u), cs, nx, ny, nz, out);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p,
                       v, n);
    return hipGetLastError();
}

hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t st)
{
    hipLaunchKernelGGL(set_i64_kernel, dim3(1), dim3(64), 0, st, p, v);
    return hipGetLastError();
}

}  // namespace abft
