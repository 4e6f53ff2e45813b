// The fused sweep kernel: Eq.(1) for a star stencil of radius 1 or 2 (RAD), with the row
// checksum (Eq.(3)), its prediction (Theorem 1, Eq.(5)) and the mismatch test (Section 3.4)
// in the same pass.
//
// Work decomposition.  A block of NW wavefronts (4 or 8) owns TY whole rows (y0 .. y0+TY-1)
// of a slab of planes z0 .. z0+tz-1 and marches along z.  Each row belongs to LPR lanes of one
// wavefront; a lane holds NCH chunks of VEC consecutive x (16-byte accesses), so the row's
// checksum is a reduction across the row's lanes (DPP) and never needs another pass over the
// data.  The planes z-RAD .. z+RAD of the block's rows and the constant term of plane z are
// kept in registers and rotated as the block advances one plane; the next plane is loaded
// while the current one is computed.  The in-plane neighbours come from LDS: every plane step
// writes the block's TY rows plus RAD halo rows on each side (loaded cooperatively by the
// whole block) into one of two LDS plane buffers, each row padded with its RAD x-ghost values
// on each side.
#pragma once

#include <type_traits>

#include "abft_device.h"

namespace abft {

// Accumulating an fp32 sweep in fp64 (one rounding per point instead of seven) was measured
// on MI355X: the fault-free row-checksum noise only fell from 5.2e-8 to 3.2e-8 of the row sum,
// because on a smooth field the points of a row round alike and the noise approaches half an
// ulp of the values whatever the accumulation, while the sweep ran 2-10% slower (more
// registers, lower occupancy).  The fp32 chain is kept.
constexpr bool kStencilAccF64 = false;

// Sum of a row held by LPR lanes, NCH chunks of VEC values per lane: each lane adds its values
// in chunk order, then the row's lanes are reduced in a fixed order.  Every lane must call it.
template <int CS, int LPR, int NCH, int VEC, typename T>
__device__ __forceinline__ double row_sum(const T (&d)[NCH][VEC])
{
    if constexpr (CS == CS_F64) {
        double p = 0.0;
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
            for (int v = 0; v < VEC; ++v) p += (double)d[c][v];
        return segment_total<LPR>(row16_sum(p));
    } else {
        CPair p{0.f, 0.f};
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
            for (int v = 0; v < VEC; ++v) p = cpair_add1(p, (float)d[c][v]);
        return segment_total<LPR>(row16_pair(p));
    }
}

// Index-weighted row sum, sum over x of (x + 1) u(x), in fp64 (values past the row end are
// zero).  A lane holds x = c * LPR * VEC + x0 + v (x0 = sl * VEC), so its share is
// (x0 + 1) * sum(u) + LPR * VEC * sum_c c * sum_v u + sum_c sum_v v * u: compile-time factors
// except one per lane (x0 + 1, given as a double), which keeps the march's registers free.
// Every lane must call it.
template <int LPR, int NCH, int VEC, typename T>
__device__ __forceinline__ double weighted_row_sum(const T (&d)[NCH][VEC], double x0p1)
{
    double all = 0.0, byc = 0.0, byv = 0.0;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        double sc = 0.0;
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            sc += (double)d[c][v];
            if (v > 0) byv = fma((double)v, (double)d[c][v], byv);
        }
        all += sc;
        if (c > 0) byc = fma((double)c, sc, byc);
    }
    const double p = fma(x0p1, all, fma((double)(LPR * VEC), byc, byv));
    return segment_total<LPR>(row16_sum(p));
}

// The input-side check of one row (the first case in the proof of Theorem 2: a value changed
// in memory after its checksum was taken): the row's sum as read against the stored checksum,
// with the threshold test of Section 3.4.  A mismatch is remembered for the repair.
__device__ __forceinline__ void check_input_row(const SweepArgs& a, int64_t t, int z, int y,
                                                double sum_read, double stored)
{
    if (!(fabs(sum_read - stored) <= a.eps * fabs(stored))) {
        const unsigned i = atomicAdd(&a.slot->mcount, 1u);
        if (i < (unsigned)kMaxMemFlags) {
            MemFlag mf;
            mf.z = z;
            mf.y = y;
            a.slot->mrows[i] = mf;
        } else {
            atomicAdd(&a.cnt->overflow, 1ull);
        }
        atomicAdd(&a.cnt->mem_flagged, 1ull);
        emit_event(a.cnt, a.ev, a.ev_cap, t, ABFT_EV_MEM_FLAG, z, y, -1, sum_read, stored,
                   a.grid);
    }
}

// One tile (TY rows x tz planes) of one sweep, run by one block.  smem_raw is the block's
// dynamic LDS (sweep_lds_bytes).
template <typename T, int MODE, int CS, int LPR, int NCH, int VEC, int PF, int NW, int RAD>
__device__ __forceinline__ void sweep_tile(const SweepArgs& a, const int tile,
                                           unsigned char* smem_raw)
{
    static_assert(RAD == 1 || RAD == 2, "star stencils of radius 1 or 2");
    using V = VecOps<T, VEC>;
    constexpr bool kProt = MODE == MODE_PROT || MODE == MODE_PROTM;
    constexpr bool kMemChk = MODE == MODE_PROTM;  // also the input-side check (a.Wn set)
    constexpr bool kRowSum = MODE == MODE_CSUM || kProt;  // whole-row checksums
    constexpr bool kTile = MODE == MODE_TILE;             // tile-local checksums instead
    constexpr int NT = NW * 64;       // threads per block
    constexpr int RPW = 64 / LPR;     // rows per wavefront
    constexpr int TY = NW * RPW;      // rows per block
    constexpr int SEGW = LPR * VEC;   // elements of one chunk of a row
    constexpr int HMAX = (NCH * SEGW + NT * VEC - 1) / (NT * VEC);
    constexpr int PAD = VEC > RAD ? VEC : RAD;  // LDS row pad, ghosts x = -RAD..-1, nx..nx+RAD-1
    constexpr int NP = 2 * RAD + 1;             // planes z-RAD .. z+RAD in registers
    constexpr int NH = 2 * RAD;                 // halo rows per LDS plane

    T* lds = reinterpret_cast<T*>(smem_raw);
    const int64_t t = a.t_off + (a.t_base != nullptr ? *a.t_base : 0);

    const int nx = a.nx, ny = a.ny, nz = a.nz, bc = a.st.bc;
    const T g = (T)a.st.g;
    // the wavefront index is uniform across the wavefront: keep it (and what derives from it)
    // in scalar registers
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int seg = lane / LPR, sl = lane % LPR;
    const int stride = nx + 2 * PAD;  // LDS row: PAD ghosts/padding, nx values, PAD
    const int plane_elems = (TY + NH) * stride;

    const int yb = tile % a.nyb, zb = tile / a.nyb;
    const int y0 = yb * TY, z0 = zb * a.tz;
    const int z1 = min(z0 + a.tz, nz);
    const int nrows = min(TY, ny - y0);
    const int r = wave * RPW + seg;
    const int y = y0 + r;
    const bool row_ok = r < nrows;

    const T* uin = static_cast<const T*>(a.uin);
    T* uout = static_cast<T*>(a.uout);
    const T* Cp = static_cast<const T*>(a.C);
    const T cs = (T)a.c_scalar;
    const size_t pstride = (size_t)nx * (size_t)ny;
    const uint32_t mask = a.st.mask;
    // accumulation type of Eq.(1) (see kStencilAccF64)
    using Acc = typename std::conditional<sizeof(T) == 4 && kStencilAccF64, double, T>::type;
    const Acc a_c = (Acc)a.st.w[W_C];
    Acc ax[RAD][2], ay[RAD][2], az[RAD][2];  // [distance - 1][minus, plus]
#pragma unroll
    for (int d = 0; d < RAD; ++d)
#pragma unroll
        for (int sg = 0; sg < 2; ++sg) {
            ax[d][sg] = (Acc)a.st.w[w_slot(0, d + 1, sg ? 1 : -1)];
            ay[d][sg] = (Acc)a.st.w[w_slot(1, d + 1, sg ? 1 : -1)];
            az[d][sg] = (Acc)a.st.w[w_slot(2, d + 1, sg ? 1 : -1)];
        }
    const uint32_t all = RAD == 1 ? 0x7Fu : 0x1FFFu;
    const bool full = mask == all;
    auto has = [&](int slot) { return (mask >> slot) & 1u; };

    int flo = 0, fhi = 0;
    if (a.faults != nullptr && t >= 0 && t < a.fault_tmax) {
        flo = a.fault_first[t];
        fhi = a.fault_first[t + 1];
    }

    // Halo rows of the block: LDS rows 0 .. RAD-1 hold y0-RAD .. y0-1, rows RAD+nrows ..
    // RAD+nrows+RAD-1 hold y0+nrows .. y0+nrows+RAD-1 (mapped by the boundary rule).
    int hy[NH], hl[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        hl[h] = h < RAD ? h : RAD + nrows + (h - RAD);
        hy[h] = map_coord(h < RAD ? y0 - RAD + h : y0 + nrows + (h - RAD), ny, bc);
    }

    // planes z-RAD .. z+RAD and the constant term of z in use; planes ahead in flight
    T pl[NP][NCH][VEC], cc[NCH][VEC], nu[NCH][VEC], nc[NCH][VEC];
    T hc[NH][HMAX][VEC], hn[NH][HMAX][VEC];
    T nu2[PF > 1 ? NCH : 1][VEC], nc2[PF > 1 ? NCH : 1][VEC], hn2[NH][PF > 1 ? HMAX : 1][VEC];

    auto load_u = [&](T (&d)[NCH][VEC], int zz) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int x = c * SEGW + sl * VEC;
            if (row_ok && x < nx) {
                if (zz >= 0) {
                    V::load(uin + (size_t)zz * pstride + (size_t)y * nx + x, d[c]);
                } else {
#pragma unroll
                    for (int v = 0; v < VEC; ++v) d[c][v] = g;
                }
            } else {
#pragma unroll
                for (int v = 0; v < VEC; ++v) d[c][v] = T(0);
            }
        }
    };
    auto load_c = [&](T (&d)[NCH][VEC], int zz) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int x = c * SEGW + sl * VEC;
            if (row_ok && x < nx && Cp != nullptr) {
                V::load_nt(Cp + (size_t)zz * pstride + (size_t)y * nx + x, d[c]);
            } else {
#pragma unroll
                for (int v = 0; v < VEC; ++v) d[c][v] = cs;
            }
        }
    };
    auto load_halo = [&](auto& d, int zz) {
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            const int yy = hy[h];
#pragma unroll
            for (int k = 0; k < HMAX; ++k) {
                const int x = (tid + k * NT) * VEC;
                if (x < nx && yy >= 0) {
                    V::load(uin + (size_t)zz * pstride + (size_t)yy * nx + x, d[h][k]);
                } else {
#pragma unroll
                    for (int v = 0; v < VEC; ++v) d[h][k][v] = g;
                }
            }
        }
    };
    // Ghost values of one LDS row from the threads holding its first and last RAD points:
    // clamp repeats the edge value, periodic wraps, constant writes the ghost value.
    auto put_ghosts = [&](T* row, int x, const T (&d)[VEC]) {
        if constexpr (VEC >= RAD) {
            // the row's first and last RAD points sit in its first and last chunks (testing
            // chunk ends only: a per-point form costs the march some 80 scalar registers in
            // spills)
            if (x == 0) {
                if (bc == ABFT_BC_CLAMP) {
#pragma unroll
                    for (int q = 1; q <= RAD; ++q) row[-q] = d[0];
                } else if (bc == ABFT_BC_PERIODIC) {
#pragma unroll
                    for (int q = 0; q < RAD; ++q) row[nx + q] = d[q];
                } else {
#pragma unroll
                    for (int q = 1; q <= RAD; ++q) {
                        row[-q] = g;
                        row[nx - 1 + q] = g;
                    }
                }
            }
            if (x + VEC == nx) {
                if (bc == ABFT_BC_CLAMP) {
#pragma unroll
                    for (int q = 0; q < RAD; ++q) row[nx + q] = d[VEC - 1];
                } else if (bc == ABFT_BC_PERIODIC) {
#pragma unroll
                    for (int q = 1; q <= RAD; ++q) row[-q] = d[VEC - q];
                }
            }
        } else {
            // one point per chunk (VEC == 1): the points 0 .. RAD-1 and nx-RAD .. nx-1
            const int xv = x;
            if (bc == ABFT_BC_CLAMP) {
                if (xv == 0)
#pragma unroll
                    for (int q = 1; q <= RAD; ++q) row[-q] = d[0];
                if (xv == nx - 1)
#pragma unroll
                    for (int q = 0; q < RAD; ++q) row[nx + q] = d[0];
            } else if (bc == ABFT_BC_PERIODIC) {
                if (xv >= nx - RAD) row[xv - nx] = d[0];
                if (xv < RAD) row[xv + nx] = d[0];
            } else if (xv == 0) {
#pragma unroll
                for (int q = 1; q <= RAD; ++q) {
                    row[-q] = g;
                    row[nx - 1 + q] = g;
                }
            }
        }
    };

    // The prediction of every row and plane of the tile (Theorem 1, Eq.(5)) depends only on the
    // previous checksums and the constant term's, except for the x-boundary term of the input
    // row, which the march forms: the block's threads take the tile's (row, plane) pairs, rows
    // fastest, so that neighbouring threads read neighbouring checksums, and leave that partial
    // prediction in an LDS table before the march.  Their loads are issued ahead of the first
    // planes' and overlap them, so no checksum load sits in the epilogue.
    auto brow = [&](int z2, int y2) -> double {
        const int mz = map_coord(z2, nz, bc), my = map_coord(y2, ny, bc);
        if (mz < 0 || my < 0) return (double)nx * (double)g;
        return a.Bt[(size_t)mz * ny + my];
    };
    // checksum, boundary-term, input-sum, weighted-sum and partial-prediction tables: [TY][tz]
    // doubles each, after the two plane buffers (the input-sum and weighted-sum tables only
    // with the input-side check; the partial predictions then follow them)
    double* tabS = reinterpret_cast<double*>(smem_raw + (size_t)2 * plane_elems * sizeof(T));
    double* tabE = tabS + TY * a.tz;
    double* tabI = tabE + TY * a.tz;
    double* tabW = tabI + TY * a.tz;
    double* tabP = kMemChk ? tabW + TY * a.tz : tabI;
    unsigned long long nknown = 0ull;
    const int npairs = nrows * (z1 - z0);  // the tile's (row, plane) pairs
    if constexpr (kProt) {
        nknown = noise_known(a.cnt);
        for (int q = tid; q < npairs; q += NT) {
            const int rr = q % nrows, pz = q / nrows;
            const int z = z0 + pz, yy = y0 + rr;
            const size_t l = (size_t)z * ny + yy;
            const double b0 = a.Bt[l];
            double bp = a.cB[l];
            if (has(W_C)) bp += a.st.w[W_C] * b0;
#pragma unroll
            for (int d = 1; d <= RAD; ++d) {
                if (has(w_slot(0, d, -1))) bp += a.st.w[w_slot(0, d, -1)] * b0;
                if (has(w_slot(0, d, 1))) bp += a.st.w[w_slot(0, d, 1)] * b0;
            }
#pragma unroll
            for (int d = 1; d <= RAD; ++d) {
                if (has(w_slot(1, d, -1))) bp += a.st.w[w_slot(1, d, -1)] * brow(z, yy - d);
                if (has(w_slot(1, d, 1))) bp += a.st.w[w_slot(1, d, 1)] * brow(z, yy + d);
                if (has(w_slot(2, d, -1))) bp += a.st.w[w_slot(2, d, -1)] * brow(z - d, yy);
                if (has(w_slot(2, d, 1))) bp += a.st.w[w_slot(2, d, 1)] * brow(z + d, yy);
            }
            tabP[rr * a.tz + pz] = bp;
        }
    }

#pragma unroll
    for (int q = 0; q < NP; ++q) load_u(pl[q], map_coord(z0 - RAD + q, nz, bc));
    load_c(cc, z0);
    load_halo(hc, z0);
    if constexpr (PF > 1) {
        if (z0 + 1 < z1) {
            load_u(nu, map_coord(z0 + RAD + 1, nz, bc));
            load_c(nc, z0 + 1);
            load_halo(hn, z0 + 1);
        }
    }
    // the x-boundary terms: for the prediction unless they cancel exactly, and for the offline
    // record when one is kept
    const bool xt = a.st.xterms != 0;
    const bool keep_e = (kProt && xt) || a.E != nullptr;
    // With one plane ahead, radius 2 issues the next plane's constant term after the plane's
    // points are stored rather than with the next plane's loads: measured, its protected sweep
    // went from 12% over the plain one to 1-2% (the plain one lost 2%); at radius 1 the
    // earlier load is kept (the later one cost small grids and batches 2-3%).
    constexpr bool kLateC = RAD == 2;

    for (int z = z0; z < z1; ++z) {
        if constexpr (kMemChk) {
            // the input row as this sweep reads it, summed like an output row (the stored
            // checksum it is compared with after the march was formed the same way); done
            // before the next planes are in flight, when the fewest registers are live
            const double Si = row_sum<CS, LPR, NCH, VEC>(pl[RAD]);
            if (row_ok && sl == 0) tabI[r * a.tz + (z - z0)] = Si;
        }
        // planes ahead in flight while this one is computed
        if constexpr (PF > 1) {
            if (z + 2 < z1) {
                load_u(nu2, map_coord(z + RAD + 2, nz, bc));
                load_c(nc2, z + 2);
                load_halo(hn2, z + 2);
            }
        } else {
            if (z + 1 < z1) {
                load_u(nu, map_coord(z + RAD + 1, nz, bc));
                if constexpr (!kLateC) load_c(nc, z + 1);
                load_halo(hn, z + 1);
            }
        }

        T* buf = lds + ((z - z0) & 1) * plane_elems;
        if (row_ok) {
            T* row = buf + (r + RAD) * stride + PAD;
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int x = c * SEGW + sl * VEC;
                if (x < nx) {
                    V::store(row + x, pl[RAD][c]);
                    put_ghosts(row, x, pl[RAD][c]);
                }
            }
        }
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            T* row = buf + hl[h] * stride + PAD;
#pragma unroll
            for (int k = 0; k < HMAX; ++k) {
                const int x = (tid + k * NT) * VEC;
                if (x < nx) {
                    V::store(row + x, hc[h][k]);
                    put_ghosts(row, x, hc[h][k]);
                }
            }
        }
        __syncthreads();

        // Eq.(1) on the block's rows of plane z.
        const T* row0 = buf + (r + RAD) * stride + PAD;
        T o[NCH][VEC];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int x = c * SEGW + sl * VEC;
            if (row_ok && x < nx) {
                T ym[RAD][VEC], yp[RAD][VEC], xlo[RAD], xhi[RAD];
#pragma unroll
                for (int d = 0; d < RAD; ++d) {
                    V::load(row0 - (d + 1) * stride + x, ym[d]);
                    V::load(row0 + (d + 1) * stride + x, yp[d]);
                    xlo[d] = row0[x - 1 - d];    // x - 1 - d
                    xhi[d] = row0[x + VEC + d];  // x + VEC + d
                }
                // the value at x + v + dx for |dx| <= RAD: this lane's chunk, else LDS
                auto xval = [&](int v, int dx) -> T {
                    const int idx = v + dx;
                    if (idx >= 0 && idx < VEC) return pl[RAD][c][idx];
                    return idx < 0 ? xlo[-idx - 1] : xhi[idx - VEC];
                };
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    Acc acc = (Acc)cc[c][v];
                    if (full) {
                        acc = fma(a_c, (Acc)pl[RAD][c][v], acc);
#pragma unroll
                        for (int d = 0; d < RAD; ++d) {
                            acc = fma(ax[d][0], (Acc)xval(v, -d - 1), acc);
                            acc = fma(ax[d][1], (Acc)xval(v, d + 1), acc);
                            acc = fma(ay[d][0], (Acc)ym[d][v], acc);
                            acc = fma(ay[d][1], (Acc)yp[d][v], acc);
                            acc = fma(az[d][0], (Acc)pl[RAD - d - 1][c][v], acc);
                            acc = fma(az[d][1], (Acc)pl[RAD + d + 1][c][v], acc);
                        }
                    } else {
                        // absent taps contribute nothing, also next to non-finite values
                        acc = fma(a_c, has(W_C) ? (Acc)pl[RAD][c][v] : Acc(0), acc);
#pragma unroll
                        for (int d = 0; d < RAD; ++d) {
                            acc = fma(ax[d][0], has(w_slot(0, d + 1, -1)) ? (Acc)xval(v, -d - 1) : Acc(0), acc);
                            acc = fma(ax[d][1], has(w_slot(0, d + 1, 1)) ? (Acc)xval(v, d + 1) : Acc(0), acc);
                            acc = fma(ay[d][0], has(w_slot(1, d + 1, -1)) ? (Acc)ym[d][v] : Acc(0), acc);
                            acc = fma(ay[d][1], has(w_slot(1, d + 1, 1)) ? (Acc)yp[d][v] : Acc(0), acc);
                            acc = fma(az[d][0], has(w_slot(2, d + 1, -1)) ? (Acc)pl[RAD - d - 1][c][v] : Acc(0), acc);
                            acc = fma(az[d][1], has(w_slot(2, d + 1, 1)) ? (Acc)pl[RAD + d + 1][c][v] : Acc(0), acc);
                        }
                    }
                    o[c][v] = (T)acc;
                }
            } else {
#pragma unroll
                for (int v = 0; v < VEC; ++v) o[c][v] = T(0);
            }
        }

        // Fault model of Section 5.1: flip a bit of the value after the update, before the
        // store; the checksum below sees the stored value.
        for (int f = flo; f < fhi; ++f) {
            const abft_fault F = a.faults[f];
            if (F.kind == ABFT_FAULT_STORE && F.attempt == a.attempt && F.grid == a.grid &&
                F.z == z && F.y == y && row_ok) {
#pragma unroll
                for (int c = 0; c < NCH; ++c)
#pragma unroll
                    for (int v = 0; v < VEC; ++v)
                        if (c * SEGW + sl * VEC + v == F.x) {
                            if constexpr (sizeof(T) == 4) {
                                o[c][v] = __builtin_bit_cast(
                                    T, __builtin_bit_cast(uint32_t, o[c][v]) ^ (1u << F.bit));
                            } else {
                                o[c][v] = __builtin_bit_cast(
                                    T, __builtin_bit_cast(uint64_t, o[c][v]) ^ (1ull << F.bit));
                            }
                        }
            }
        }

        if (row_ok) {
            T* dst = uout + (size_t)z * pstride + (size_t)y * nx;
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int x = c * SEGW + sl * VEC;
                if (x < nx) V::store_nt(dst + x, o[c]);
            }
        }
        if constexpr (PF == 1 && kLateC) {
            // the next plane's constant term, loaded once this plane's points are done
            if (z + 1 < z1) load_c(nc, z + 1);
        }

        // Row checksum of the output (Eq.(3)), reduced across the row's lanes, and the row's
        // x-boundary term of Theorem 1 from the input row (its first and last RAD points and
        // the ghosts).  Both go to a small LDS table; the prediction and the comparison for
        // all planes of the tile run after the march, so none of their loads sits in this loop.
        if constexpr (kRowSum) {
            const double S = row_sum<CS, LPR, NCH, VEC>(o);
            if (row_ok && sl == 0) tabS[r * a.tz + (z - z0)] = S;
        }
        if constexpr (kTile) {
            // Tile-local checksums: a tile is the 16 * VEC consecutive points one 16-lane group
            // holds of a chunk.  Its output sum (a 16-lane reduction) and its x-boundary term
            // of Theorem 1 on the tile as a sub-domain, from the input row in LDS: a shift
            // dx < 0 brings in the points before the tile (a neighbouring tile's, or ghosts)
            // and drops its last |dx|; dx > 0 brings in the points after it and drops its first
            // dx.  The group's first lane forms the terms at the tile's start, its last lane
            // those at the end, and a row mirror adds them.  The prediction and the comparison
            // run in a separate launch over all tiles.
            constexpr int TT = 16 * VEC;
            const int g16 = sl & 15;
            const int ntx = nx / TT;
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                double p = 0.0;
#pragma unroll
                for (int v = 0; v < VEC; ++v) p += (double)o[c][v];
                const double ts = row16_sum(p);
                const int x0 = c * SEGW + (sl - g16) * VEC;
                double ep = 0.0;
                if (row_ok && x0 < nx && (g16 == 0 || g16 == 15)) {
#pragma unroll
                    for (int d = 1; d <= RAD; ++d) {
                        const double wm = has(w_slot(0, d, -1)) ? a.st.w[w_slot(0, d, -1)] : 0.0;
                        const double wp = has(w_slot(0, d, 1)) ? a.st.w[w_slot(0, d, 1)] : 0.0;
                        double in_m = 0.0, out_m = 0.0, in_p = 0.0, out_p = 0.0;
                        if (g16 == 0) {
#pragma unroll
                            for (int q = 1; q <= d; ++q) in_m += (double)row0[x0 - q];
#pragma unroll
                            for (int q = 0; q < d; ++q) out_p += (double)row0[x0 + q];
                        } else {
#pragma unroll
                            for (int q = 0; q < d; ++q) in_p += (double)row0[x0 + TT + q];
#pragma unroll
                            for (int q = 1; q <= d; ++q) out_m += (double)row0[x0 + TT - q];
                        }
                        ep += wm * (in_m - out_m) + wp * (in_p - out_p);
                    }
                }
                const double e = ep + dpp_d<DPP_ROW_MIRROR>(ep);
                if (row_ok && x0 < nx && g16 == 0) {
                    const size_t lt = ((size_t)z * ny + y) * ntx + x0 / TT;
                    a.Bn[lt] = ts;
                    a.Et[lt] = e;
                }
            }
        }
        if (kMemChk || (MODE == MODE_CSUM && a.Wn != nullptr)) {
            // the index-weighted sum of the output row, which places a changed point later
            // (with the input-side check; offline, for the checkpoint the window ends on)
            const double Sw = weighted_row_sum<LPR, NCH, VEC>(o, (double)(sl * VEC + 1));
            if (row_ok && sl == 0) tabW[r * a.tz + (z - z0)] = Sw;
        }
        if (keep_e && row_ok && sl == 0) {
            // shift dx < 0 reads G(dx .. -1) and drops u(nx+dx .. nx-1); dx > 0 reads
            // G(nx .. nx+dx-1) and drops u(0 .. dx-1)
            double e = 0.0;
#pragma unroll
            for (int d = 1; d <= RAD; ++d) {
                if (has(w_slot(0, d, -1))) {
                    double b = 0.0;
                    for (int q = 1; q <= d; ++q) b += (double)row0[-q] - (double)row0[nx - q];
                    e += a.st.w[w_slot(0, d, -1)] * b;
                }
                if (has(w_slot(0, d, 1))) {
                    double b = 0.0;
                    for (int q = 0; q < d; ++q) b += (double)row0[nx + q] - (double)row0[q];
                    e += a.st.w[w_slot(0, d, 1)] * b;
                }
            }
            tabE[r * a.tz + (z - z0)] = e;
        }

        // rotate the register planes
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
#pragma unroll
                for (int q = 0; q < NP - 1; ++q) pl[q][c][v] = pl[q + 1][c][v];
                pl[NP - 1][c][v] = nu[c][v];
                cc[c][v] = nc[c][v];
                if constexpr (PF > 1) {
                    nu[c][v] = nu2[c][v];
                    nc[c][v] = nc2[c][v];
                }
            }
#pragma unroll
        for (int h = 0; h < NH; ++h)
#pragma unroll
            for (int k = 0; k < HMAX; ++k)
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    hc[h][k][v] = hn[h][k][v];
                    if constexpr (PF > 1) hn[h][k][v] = hn2[h][k][v];
                }
    }

    if constexpr (!kRowSum) {
        if (a.E == nullptr) return;
    }
    __syncthreads();
    // Epilogue: the block's threads take the tile's (row, plane) pairs, rows fastest, as before
    // the march.
    double noise = 0.0;
    {
        for (int q = tid; q < npairs; q += NT) {
            const int r = q % nrows, pz = q / nrows;
            const int z = z0 + pz, y = y0 + r;
            const size_t l = (size_t)z * ny + y;
            if (a.E != nullptr) a.E[l] = tabE[r * a.tz + pz];
            if constexpr (kRowSum) {
                const double S = tabS[r * a.tz + pz];
                a.Bn[l] = S;
                if constexpr (MODE == MODE_CSUM) {
                    if (a.Wn != nullptr) a.Wn[l] = tabW[r * a.tz + pz];
                }
                if constexpr (kProt) {
                    // Theorem 1 (Eq.(5)) on the checksum plane: the partial prediction formed
                    // before the march, plus the x-boundary term of the input row
                    double bp = tabP[r * a.tz + pz];
                    if (xt) bp += tabE[r * a.tz + pz];
                    if constexpr (kMemChk) {
                        a.Wn[l] = tabW[r * a.tz + pz];
                        check_input_row(a, t, z, y, tabI[r * a.tz + pz], a.Bt[l]);
                    }
                    // Section 3.4, written so that NaN and Inf mismatches are flagged
                    const double dlt = fabs(S - bp);
                    if (!(dlt <= a.eps * fabs(bp))) {
                        const unsigned i = atomicAdd(&a.slot->count, 1u);
                        if (i < (unsigned)kMaxFlags) {
                            RowFlag rf;
                            rf.z = z;
                            rf.y = y;
                            rf.k = 0;
                            rf.pad = 0;
                            rf.direct = S;
                            rf.pred = bp;
                            a.slot->rows[i] = rf;
                        } else {
                            atomicAdd(&a.cnt->overflow, 1ull);
                        }
                        atomicAdd(&a.cnt->rows_flagged, 1ull);
                        emit_event(a.cnt, a.ev, a.ev_cap, t, ABFT_EV_ROW_FLAG, z, y, -1, S, bp,
                                   a.grid);
                    } else if (bp != 0.0) {
                        noise = fmax(noise, dlt / fabs(bp));
                    }
                }
            }
        }
    }
    if constexpr (kProt) record_noise(a.cnt, noise, nknown);
}

template <typename T, int MODE, int CS, int LPR, int NCH, int VEC, int PF, int NW, int RAD>
__global__ void __launch_bounds__(NW * 64) sweep_kernel(const SweepArgs a)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    if (a.guard != nullptr && *a.guard == 0u) return;
    const int nt = a.ntiles, bid = blockIdx.x;
    if (a.zero_ptr != nullptr && bid == 0 && (int)threadIdx.x < a.zero_n)
        a.zero_ptr[threadIdx.x] = 0u;
    // Blocks are dealt to the 8 XCDs round-robin; give each XCD a contiguous run of tiles so
    // that neighbouring row blocks (which share halo rows) meet in the same L2.
    const int per = nt >> 3, rem = nt & 7, xcd = bid & 7, q = bid >> 3;
    const int tile = xcd * per + (xcd < rem ? xcd : rem) + q;
    sweep_tile<T, MODE, CS, LPR, NCH, VEC, PF, NW, RAD>(a, tile, smem_raw);
}

// Table of instantiated variants (radius 2: prefetch depth 1 only).
template <typename T, int MODE, int CS, int RAD>
hipError_t launch_sweep_t(const SweepShape& s, const SweepArgs& a, hipStream_t st, size_t lds)
{
#define ABFT_SWEEP_CASE_NW(LPR_, NCH_, VEC_, PF_, NW_)                                        \
    if (s.lpr == LPR_ && s.nch == NCH_ && s.vec == VEC_ && s.pf == PF_ && s.nw == NW_) {       \
        auto kern = sweep_kernel<T, MODE, CS, LPR_, NCH_, VEC_, PF_, NW_, RAD>;                \
        static LdsAllowed lds_ok;                                                              \
        if (hipError_t e = allow_lds(reinterpret_cast<const void*>(kern), lds, lds_ok))        \
            return e;                                                                          \
        hipLaunchKernelGGL(kern, dim3(a.ntiles), dim3(NW_ * 64), lds, st, a);                  \
        return hipGetLastError();                                                              \
    }
// Blocks of 8 wavefronts only where a lane's share of a row is at most 64 bytes: with more,
// the planes held in registers exceed the 256 registers a lane may have at that block size.
// At radius 2 (five planes) the 64-byte shapes take 230-234 registers without spilling.
#define ABFT_SWEEP_CASE_PF(LPR_, NCH_, VEC_, PF_)                                              \
    ABFT_SWEEP_CASE_NW(LPR_, NCH_, VEC_, PF_, 4)                                               \
    if constexpr (NCH_ * VEC_ * sizeof(T) <= kWideBlockLaneBytes) {                            \
        ABFT_SWEEP_CASE_NW(LPR_, NCH_, VEC_, PF_, 8)                                           \
    }
#define ABFT_SWEEP_CASE(LPR_, NCH_, VEC_) ABFT_SWEEP_CASE_PF(LPR_, NCH_, VEC_, 1)
    constexpr int VF = 16 / (int)sizeof(T);
    if constexpr (RAD == 1) {
        ABFT_SWEEP_CASE_PF(64, 2, VF, 2)
        ABFT_SWEEP_CASE_PF(64, 4, VF, 2)
    }
    ABFT_SWEEP_CASE(16, 1, VF)
    ABFT_SWEEP_CASE(16, 2, VF)
    ABFT_SWEEP_CASE(16, 4, VF)
    ABFT_SWEEP_CASE(64, 1, VF)
    ABFT_SWEEP_CASE(64, 2, VF)
    ABFT_SWEEP_CASE(64, 4, VF)
    ABFT_SWEEP_CASE(64, 8, VF)
    if constexpr (MODE != MODE_TILE) {  // tiles are 16 lanes of 16-byte accesses
        ABFT_SWEEP_CASE(64, 4, 1)
        ABFT_SWEEP_CASE(64, 16, 1)
    }
#undef ABFT_SWEEP_CASE
#undef ABFT_SWEEP_CASE_PF
#undef ABFT_SWEEP_CASE_NW
    return hipErrorInvalidValue;
}

}  // namespace abft
