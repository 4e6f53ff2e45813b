// The fused sweep for 27-point box stencils (every tap (dx, dy, dz) with offsets in -1..1),
// with the row checksum (Eq.(3)), its prediction (Theorem 1) and the mismatch test
// (Section 3.4) in the same pass.
//
// The decomposition is that of the star sweep (abft_sweep.h): a block of NW wavefronts owns
// TY whole rows of a slab of planes and marches along z, each row held by LPR lanes.  A box
// tap reads the in-plane neighbours of planes z-1 and z+1 as well.  The march visits each input
// plane p once: it goes through LDS (the block's rows, one halo row above and below, the
// x-ghosts), each lane gathers its 3 x 3 in-plane neighbourhood from there once, and the nine
// values feed three accumulators held in registers, those of output planes p+1 (taps dz = -1),
// p (dz = 0) and p-1 (dz = +1), which is then complete.  Every output so receives its taps in
// the order dz, dy, dx.  Two LDS plane buffers alternate: plane p+1 is written into the one
// plane p-1 used, after the step's single barrier.
//
// Theorem 1 for a box stencil: the row sum of the output row (z, y) is the constant term's
// row sum plus, for every (dy, dz), the weight sum over dx times the input row sum of row
// (z+dz, y+dy), plus the x-boundary terms of those nine rows (their ghost values minus the
// points a shift drops), weighted by the dx = -1 and dx = +1 taps.  The nine rows are in LDS
// at step z, so the boundary terms are formed in the march; the row sums of the input come
// from the previous sweep's checksum plane in the epilogue.
#pragma once

#include "abft_sweep.h"

namespace abft {

template <typename T, int MODE, int CS, int LPR, int NCH, int VEC, int NW>
__device__ __forceinline__ void sweep_box_tile(const SweepArgs& a, const int tile,
                                               unsigned char* smem_raw)
{
    using V = VecOps<T, VEC>;
    constexpr bool kProt = MODE == MODE_PROT || MODE == MODE_PROTM;
    constexpr bool kMemChk = MODE == MODE_PROTM;  // also the input-side check (a.Wn set)
    constexpr int NT = NW * 64;
    constexpr int RPW = 64 / LPR;
    constexpr int TY = NW * RPW;
    constexpr int SEGW = LPR * VEC;
    constexpr int HMAX = (NCH * SEGW + NT * VEC - 1) / (NT * VEC);
    constexpr int NB = 2;  // LDS plane buffers, alternating

    T* lds = reinterpret_cast<T*>(smem_raw);
    const int64_t t = a.t_off + (a.t_base != nullptr ? *a.t_base : 0);
    const int nx = a.nx, ny = a.ny, nz = a.nz, bc = a.st.bc;
    const T g = (T)a.st.g;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int seg = lane / LPR, sl = lane % LPR;
    const int stride = nx + 2 * VEC;
    const int plane_elems = (TY + 2) * stride;

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
    const uint32_t bmask = a.st.bmask;
    auto has = [&](int slot) { return (bmask >> slot) & 1u; };
    // every tap present: the march needs no per-point selection of the absent ones
    const bool full = bmask == 0x7FFFFFFu;
    T wt[27];  // the weights in the grid dtype, converted once
#pragma unroll
    for (int k = 0; k < 27; ++k) wt[k] = (T)a.st.wb[k];

    int flo = 0, fhi = 0;
    if (a.faults != nullptr && t >= 0 && t < a.fault_tmax) {
        flo = a.fault_first[t];
        fhi = a.fault_first[t + 1];
    }
    const int yh0 = map_coord(y0 - 1, ny, bc), yh1 = map_coord(y0 + nrows, ny, bc);
    const int lh1 = nrows + 1;

    T nu[NCH][VEC], cn[NCH][VEC];  // the next input plane's rows, the next output's C
    T hn[2][HMAX][VEC];

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
    auto load_halo = [&](T (&d)[2][HMAX][VEC], int zz) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int yy = h ? yh1 : yh0;
#pragma unroll
            for (int k = 0; k < HMAX; ++k) {
                const int x = (tid + k * NT) * VEC;
                if (x < nx && yy >= 0 && zz >= 0) {
                    V::load(uin + (size_t)zz * pstride + (size_t)yy * nx + x, d[h][k]);
                } else {
#pragma unroll
                    for (int v = 0; v < VEC; ++v) d[h][k][v] = g;
                }
            }
        }
    };
    auto put_ghosts = [&](T* row, int x, const T (&d)[VEC]) {
        if (x == 0) {
            if (bc == ABFT_BC_CLAMP) row[-1] = d[0];
            else if (bc == ABFT_BC_PERIODIC) row[nx] = d[0];
            else { row[-1] = g; row[nx] = g; }
        }
        if (x + VEC == nx) {
            if (bc == ABFT_BC_CLAMP) row[nx] = d[VEC - 1];
            else if (bc == ABFT_BC_PERIODIC) row[-1] = d[VEC - 1];
        }
    };
    // A plane (the rows loaded for it, constant ghosts for a plane outside the grid) into LDS
    // buffer b.
    auto buf_of = [&](int b) { return lds + (b % NB) * plane_elems; };
    auto put_plane = [&](T* buf, const T (&own)[NCH][VEC], const T (&hal)[2][HMAX][VEC]) {
        if (row_ok) {
            T* row = buf + (r + 1) * stride + VEC;
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int x = c * SEGW + sl * VEC;
                if (x < nx) {
                    V::store(row + x, own[c]);
                    put_ghosts(row, x, own[c]);
                }
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            T* row = buf + (h ? lh1 : 0) * stride + VEC;
#pragma unroll
            for (int k = 0; k < HMAX; ++k) {
                const int x = (tid + k * NT) * VEC;
                if (x < nx) {
                    V::store(row + x, hal[h][k]);
                    put_ghosts(row, x, hal[h][k]);
                }
            }
        }
    };

    auto brow = [&](int z2, int y2) -> double {
        const int mz = map_coord(z2, nz, bc), my = map_coord(y2, ny, bc);
        if (mz < 0 || my < 0) return (double)nx * (double)g;
        return a.Bt[(size_t)mz * ny + my];
    };
    unsigned long long nknown = 0ull;

    // prologue: plane z0-1 into buffer 0; plane z0 and the constant term of output z0 in flight
    {
        T pu[NCH][VEC], ph[2][HMAX][VEC];
        load_u(pu, map_coord(z0 - 1, nz, bc));
        load_halo(ph, map_coord(z0 - 1, nz, bc));
        put_plane(buf_of(0), pu, ph);
    }
    load_u(nu, z0);
    load_halo(hn, z0);
    load_c(cn, z0);

    // the boundary terms: lane j < 9 of a row takes, at each step, the row y + ldy of the
    // plane in LDS, for the output ldz planes before it; its weights
    const int ldz = sl / 3 - 1, ldy = sl % 3 - 1;
    double lwm = 0.0, lwp = 0.0;
    bool lhm = false, lhp = false;
    if (sl < 9) {
        const int sm = box_slot(-1, ldy, ldz), sp = box_slot(1, ldy, ldz);
        lhm = has(sm);
        lhp = has(sp);
        lwm = a.st.wb[sm];
        lwp = a.st.wb[sp];
    }

    double* tabS = reinterpret_cast<double*>(smem_raw + (size_t)NB * plane_elems * sizeof(T));
    double* tabE = tabS + TY * a.tz;
    double* tabI = tabE + TY * a.tz;
    double* tabW = tabI + TY * a.tz;
    double* tabP = kMemChk ? tabW + TY * a.tz : tabI;  // partial predictions
    // The prediction of every row and plane of the tile (Theorem 1 for the box: the weight sums
    // over dx times the nine input row sums, plus the constant term's) except the boundary
    // terms the march forms, by the block's threads over the tile's (row, plane) pairs, rows
    // fastest, into an LDS table; the loads overlap those of the planes in flight.
    const int npairs = nrows * (z1 - z0);
    if constexpr (kProt) {
        nknown = noise_known(a.cnt);
        for (int q = tid; q < npairs; q += NT) {
            const int rr = q % nrows, pz = q / nrows;
            const int z = z0 + pz, yy = y0 + rr;
            double bp = a.cB[(size_t)z * ny + yy];
#pragma unroll
            for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
                for (int dy = -1; dy <= 1; ++dy) {
                    double wsum = 0.0;
                    bool any = false;
#pragma unroll
                    for (int dx = -1; dx <= 1; ++dx) {
                        const int sl_ = box_slot(dx, dy, dz);
                        if (has(sl_)) {
                            wsum += a.st.wb[sl_];
                            any = true;
                        }
                    }
                    if (any) bp += wsum * brow(z + dz, yy + dy);
                }
            tabP[rr * a.tz + pz] = bp;
        }
    }
    // the x-boundary terms: for the prediction unless they cancel exactly, and for the offline
    // record when one is kept
    const bool xt = a.st.xterms != 0;
    const bool keep_e = (kProt && xt) || a.E != nullptr;
    using Acc = T;

    T acc[3][NCH][VEC];  // at step p: the accumulators of outputs p-1, p, p+1
    const int nsteps = z1 - z0 + 2;
    for (int st = 0; st < nsteps; ++st) {
        const int p = z0 - 1 + st;  // the input plane of this step
        __syncthreads();  // plane p is in its buffer; the reads of the other one are over
        // plane p+1 into the other buffer, and output p+1 starts from its constant term.  The
        // loads ahead are not conditional on the step (near the slab's end they repeat its last
        // plane), so that no register copy has to wait for them.
        put_plane(buf_of(st + 1), nu, hn);
        load_u(nu, map_coord(min(p + 2, z1), nz, bc));
        load_halo(hn, map_coord(min(p + 2, z1), nz, bc));
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[2][c][v] = (Acc)cn[c][v];
        const T* prow = buf_of(st) + (r + 1) * stride + VEC;  // row y of plane p in LDS

#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int x = c * SEGW + sl * VEC;
            if (row_ok && x < nx) {
                // each in-plane neighbour once, into the three outputs it is a tap of (tap
                // (dx, dy, dz) of output p - dz); absent taps contribute nothing, also next to
                // non-finite values; with every tap present, no per-point selection
                auto taps = [&](auto every) {
                    constexpr bool kEvery = decltype(every)::value;
#pragma unroll
                    for (int dy = -1; dy <= 1; ++dy) {
                        const T* rw = prow + dy * stride;
                        T m[VEC];
                        V::load(rw + x, m);
                        const T xl = rw[x - 1], xr = rw[x + VEC];
#pragma unroll
                        for (int dx = -1; dx <= 1; ++dx)
#pragma unroll
                            for (int dz = -1; dz <= 1; ++dz) {
                                const int sl_ = box_slot(dx, dy, dz);
                                const Acc wv = (Acc)wt[sl_];
                                const bool on = kEvery || has(sl_);
#pragma unroll
                                for (int v = 0; v < VEC; ++v) {
                                    const int idx = v + dx;
                                    const T val = idx < 0 ? xl : (idx >= VEC ? xr : m[idx]);
                                    acc[1 - dz][c][v] =
                                        fma(wv, on ? (Acc)val : Acc(0), acc[1 - dz][c][v]);
                                }
                            }
                    }
                };
                if (full) taps(std::true_type{});
                else taps(std::false_type{});
            }
        }

        if constexpr (kMemChk) {
            // the input row (p, y) as read (from LDS), for the input-side check
            if (p >= z0 && p < z1) {
                T ci[NCH][VEC];
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    const int x = c * SEGW + sl * VEC;
                    if (row_ok && x < nx) {
                        V::load(prow + x, ci[c]);
                    } else {
#pragma unroll
                        for (int v = 0; v < VEC; ++v) ci[c][v] = T(0);
                    }
                }
                const double Si = row_sum<CS, LPR, NCH, VEC>(ci);
                if (row_ok && sl == 0) tabI[r * a.tz + (p - z0)] = Si;
            }
        }
        if (keep_e) {
            // x-boundary terms of the input row (p, y + ldy) for output p - ldz: a shift
            // dx = -1 reads G(-1) and drops u(nx-1); dx = +1 reads G(nx) and drops u(0).  Per
            // output, a 16-lane reduction sums its three rows of plane p.
            double part = 0.0;
            if (row_ok && sl < 9) {
                const T* rw = prow + ldy * stride;
                if (lhm) part += lwm * ((double)rw[-1] - (double)rw[nx - 1]);
                if (lhp) part += lwp * ((double)rw[nx] - (double)rw[0]);
            }
#pragma unroll
            for (int k = -1; k <= 1; ++k) {
                const double e = row16_sum(ldz == k ? part : 0.0);
                const int zo = p - k;
                if (zo >= z0 && zo < z1 && row_ok && sl == 0) {
                    double& te = tabE[r * a.tz + (zo - z0)];
                    te = k == -1 ? e : te + e;
                }
            }
        }

        load_c(cn, min(p + 2, z1 - 1));  // after the gather, so that it holds no registers there

        // output p-1 is complete
        const int z = p - 1;
        if (z >= z0) {
            T o[NCH][VEC];
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const bool ok = row_ok && c * SEGW + sl * VEC < nx;
#pragma unroll
                for (int v = 0; v < VEC; ++v) o[c][v] = ok ? (T)acc[0][c][v] : T(0);
            }

            // Fault model of Section 5.1 (as in the star sweep).
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
                                        T, __builtin_bit_cast(uint64_t, o[c][v]) ^
                                               (1ull << F.bit));
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

            if constexpr (MODE != MODE_PLAIN) {
                const double S = row_sum<CS, LPR, NCH, VEC>(o);
                if (row_ok && sl == 0) tabS[r * a.tz + (z - z0)] = S;
            }
            if constexpr (kMemChk) {
                // the output's index-weighted sum, as in the star sweep
                const double Sw = weighted_row_sum<LPR, NCH, VEC>(o, (double)(sl * VEC + 1));
                if (row_ok && sl == 0) tabW[r * a.tz + (z - z0)] = Sw;
            }
            if constexpr (MODE == MODE_CSUM) {
                if (a.Wn != nullptr) {  // offline: the weighted sums of the checkpoint to be
                    const double Sw = weighted_row_sum<LPR, NCH, VEC>(o, (double)(sl * VEC + 1));
                    if (row_ok && sl == 0) tabW[r * a.tz + (z - z0)] = Sw;
                }
            }
        }
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                acc[0][c][v] = acc[1][c][v];
                acc[1][c][v] = acc[2][c][v];
            }
    }

    if constexpr (MODE == MODE_PLAIN) {
        if (a.E == nullptr) return;
    }
    __syncthreads();
    // the block's threads take the tile's (row, plane) pairs, rows fastest
    double noise = 0.0;
    {
        for (int q = tid; q < npairs; q += NT) {
            const int r = q % nrows, pz = q / nrows;
            const int z = z0 + pz, y = y0 + r;
            const size_t l = (size_t)z * ny + y;
            if (a.E != nullptr) a.E[l] = tabE[r * a.tz + pz];
            if constexpr (MODE != MODE_PLAIN) {
                const double S = tabS[r * a.tz + pz];
                a.Bn[l] = S;
                if constexpr (MODE == MODE_CSUM) {
                    if (a.Wn != nullptr) a.Wn[l] = tabW[r * a.tz + pz];
                }
                if constexpr (kProt) {
                    // Theorem 1 for the box: the partial prediction formed before the march,
                    // plus the boundary terms formed in it
                    double bp = tabP[r * a.tz + pz];
                    if (xt) bp += tabE[r * a.tz + pz];
                    if constexpr (kMemChk) {
                        a.Wn[l] = tabW[r * a.tz + pz];
                        check_input_row(a, t, z, y, tabI[r * a.tz + pz], a.Bt[l]);
                    }
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

template <typename T, int MODE, int CS, int LPR, int NCH, int VEC, int NW>
__global__ void __launch_bounds__(NW * 64) sweep_box_kernel(const SweepArgs a)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    if (a.guard != nullptr && *a.guard == 0u) return;
    const int nt = a.ntiles, bid = blockIdx.x;
    if (a.zero_ptr != nullptr && bid == 0 && (int)threadIdx.x < a.zero_n)
        a.zero_ptr[threadIdx.x] = 0u;
    const int per = nt >> 3, rem = nt & 7, xcd = bid & 7, q = bid >> 3;
    const int tile = xcd * per + (xcd < rem ? xcd : rem) + q;
    sweep_box_tile<T, MODE, CS, LPR, NCH, VEC, NW>(a, tile, smem_raw);
}

// Table of instantiated box variants (prefetch depth 1).
template <typename T, int MODE, int CS>
hipError_t launch_sweep_box_t(const SweepShape& s, const SweepArgs& a, hipStream_t st,
                              size_t lds)
{
#define ABFT_BOX_CASE_NW(LPR_, NCH_, VEC_, NW_)                                               \
    if (s.lpr == LPR_ && s.nch == NCH_ && s.vec == VEC_ && s.nw == NW_) {                      \
        auto kern = sweep_box_kernel<T, MODE, CS, LPR_, NCH_, VEC_, NW_>;                      \
        static LdsAllowed lds_ok;                                                              \
        if (hipError_t e = allow_lds(reinterpret_cast<const void*>(kern), lds, lds_ok))        \
            return e;                                                                          \
        hipLaunchKernelGGL(kern, dim3(a.ntiles), dim3(NW_ * 64), lds, st, a);                  \
        return hipGetLastError();                                                              \
    }
#define ABFT_BOX_CASE(LPR_, NCH_, VEC_)                                                        \
    ABFT_BOX_CASE_NW(LPR_, NCH_, VEC_, 4)                                                      \
    if constexpr (NCH_ * VEC_ * sizeof(T) <= kWideBlockLaneBytes) {                            \
        ABFT_BOX_CASE_NW(LPR_, NCH_, VEC_, 8)                                                  \
    }
    constexpr int VF = 16 / (int)sizeof(T);
    ABFT_BOX_CASE(16, 1, VF)
    ABFT_BOX_CASE(16, 2, VF)
    ABFT_BOX_CASE(16, 4, VF)
    ABFT_BOX_CASE(64, 1, VF)
    ABFT_BOX_CASE(64, 2, VF)
    ABFT_BOX_CASE(64, 4, VF)
    ABFT_BOX_CASE(64, 8, VF)
    ABFT_BOX_CASE(64, 4, 1)
    ABFT_BOX_CASE(64, 16, 1)
#undef ABFT_BOX_CASE
#undef ABFT_BOX_CASE_NW
    return hipErrorInvalidValue;
}

}  // namespace abft
