// The batched sweep kernel: many independent grids of uneven sizes swept by one launch.
//
// The tiles of all grids form one list, largest first.  In the persistent form a fixed grid of
// blocks (enough to fill the compute units once) pops tiles from an atomic counter, fetching
// the next index while the current tile runs; in the direct form block b takes tile b and the
// hardware dispatcher does the balancing.  Every tile runs the same fused sweep/checksum code
// as a single grid (sweep_tile, or sweep_box_tile for box stencils), with that grid's
// descriptor; all grids of a batch share the stencil form (radius and box), each has its own
// weights.  Blocks of 4 wavefronts loading one plane ahead (8 wavefronts or two planes ahead
// were slower on batches of small grids).
#pragma once

#include "abft_box.h"

namespace abft {

// A value that no lane writes during the launch, read through the constant address space: with
// a uniform address the load is scalar and the value lives in scalar registers.
template <typename S>
__device__ __forceinline__ S load_const(const S* src)
{
    return *(const __attribute__((address_space(4))) S*)src;
}

// The plain radius-1 variant fits three wavefronts per SIMD with no spill when asked to (168
// registers instead of 172); the checksum variants would spill, and run slower, at that limit.
// NCHB, NCHC: narrower chunk counts the launch also holds (radius-1 stars only), 0 for none; a
// grid's descriptor says which of the three its rows take, so that grids of shorter rows share
// the launch without idle chunks.
template <typename T, int MODE, int CS, int LPR, int NCH, int VEC, int RAD, int BOX, int NCHB = 0,
          int NCHC = 0>
__global__ void __launch_bounds__(kBatchWaves * 64)
    __attribute__((amdgpu_waves_per_eu(MODE == MODE_PLAIN && RAD == 1 && !BOX && VEC > 1 ? 3 : 1)))
    sweep_batch_kernel(const BatchArgs b)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    __shared__ int sh_next;
    const int p = b.parity;
    if (b.zero_slots && blockIdx.x == 0) {
        // the next sweep's flag slots start from zero
        for (int g = threadIdx.x; g < b.ngrids; g += blockDim.x) {
            b.grids[g].slot[p ^ 1]->count = 0u;
            b.grids[g].slot[p ^ 1]->mcount = 0u;
        }
    }
    int it;
    if (b.persistent) {
        if (threadIdx.x == 0) sh_next = (int)atomicAdd(&b.queue[0], 1u);
        __syncthreads();
        // the index is the same in every lane: keeping it (and so the tile's descriptor) in
        // scalar registers leaves the vector registers to the sweep
        it = __builtin_amdgcn_readfirstlane(sh_next);
    } else {
        it = blockIdx.x;
    }
    while (it < b.ntiles) {
        __syncthreads();  // everyone has read sh_next; the previous tile's LDS use is over
        if (b.persistent && threadIdx.x == 0) sh_next = (int)atomicAdd(&b.queue[0], 1u);
        // the tile list and the descriptors do not change during the launch, and the index is
        // uniform: the descriptor's pointers, sizes and weights come in by scalar loads
        const int gx = load_const(&b.order[it].x), gy = load_const(&b.order[it].y);
        const GridDesc* d = b.grids + gx;
        SweepArgs a{};
        a.uin = load_const(&d->u[p]);
        a.uout = load_const(&d->u[p ^ 1]);
        a.C = load_const(&d->C);
        a.c_scalar = load_const(&d->c_scalar);
#pragma unroll
        for (int k = 0; k < W_COUNT; ++k) a.st.w[k] = load_const(&d->st.w[k]);
        a.st.mask = load_const(&d->st.mask);
        a.st.bc = load_const(&d->st.bc);
        a.st.g = load_const(&d->st.g);
        a.st.xterms = load_const(&d->st.xterms);
        a.st.rad = RAD;
        a.st.box = BOX;
        if constexpr (BOX) {
#pragma unroll
            for (int k = 0; k < 27; ++k) a.st.wb[k] = load_const(&d->st.wb[k]);
            a.st.bmask = load_const(&d->st.bmask);
        }
        a.nx = load_const(&d->nx);
        a.ny = load_const(&d->ny);
        a.nz = load_const(&d->nz);
        a.tz = load_const(&d->tz);
        a.nyb = load_const(&d->nyb);
        a.ntiles = load_const(&d->ntiles);
        a.attempt = b.attempt;
        a.t_base = b.t_base;
        a.t_off = b.t_off;
        a.Bt = load_const(&d->B[p]);
        a.Bn = load_const(&d->B[p ^ 1]);
        a.Wn = load_const(&d->W[p ^ 1]);
        a.cB = load_const(&d->cB);
        a.eps = b.eps;
        a.slot = load_const(&d->slot[p]);
        a.cnt = b.cnt;
        a.ev = b.ev;
        a.ev_cap = b.ev_cap;
        a.grid = gx;
        a.faults = b.faults;
        a.fault_first = b.fault_first;
        a.fault_tmax = b.fault_tmax;
        if constexpr (BOX) {
            sweep_box_tile<T, MODE, CS, LPR, NCH, VEC, kBatchWaves>(a, gy, smem_raw);
        } else {
            auto tile = [&](auto nch) {
                sweep_tile<T, MODE, CS, LPR, decltype(nch)::value, VEC, 1, kBatchWaves, RAD>(
                    a, gy, smem_raw);
            };
            if constexpr (NCHB > 0) {
                const int sub = load_const(&d->sub);
                if constexpr (NCHC > 0) {
                    if (sub == 2) tile(std::integral_constant<int, (NCHC > 0 ? NCHC : 1)>{});
                    else if (sub == 1) tile(std::integral_constant<int, NCHB>{});
                    else tile(std::integral_constant<int, NCH>{});
                } else {
                    if (sub == 1) tile(std::integral_constant<int, NCHB>{});
                    else tile(std::integral_constant<int, NCH>{});
                }
            } else {
                tile(std::integral_constant<int, NCH>{});
            }
        }
        if (!b.persistent) break;
        __syncthreads();
        it = __builtin_amdgcn_readfirstlane(sh_next);
    }
    if (b.persistent && threadIdx.x == 0) {
        // every block has drawn past the end of the list before it leaves, so the last one to
        // leave can rewind the counter for the next launch
        if (atomicAdd(&b.queue[1], 1u) == gridDim.x - 1) {
            atomicExch(&b.queue[0], 0u);
            atomicExch(&b.queue[1], 0u);
        }
    }
}

// Instantiated shapes, one per size class of rows: 16 lanes per row with 1, 2 or 4 chunks of
// 16-byte accesses (rows up to 64, 128, 256 fp32 points), 64 lanes with 1, 2 or 4 chunks (up to
// 256, 512, 1024), and 64 lanes of single elements for rows that are not 16-byte multiples.
#define ABFT_BATCH_SHAPES(X)                                                                   \
    constexpr int VF = 16 / (int)sizeof(T);                                                    \
    X(16, 1, VF)                                                                               \
    X(16, 2, VF)                                                                               \
    X(16, 4, VF)                                                                               \
    X(64, 1, VF)                                                                               \
    X(64, 2, VF)                                                                               \
    X(64, 4, VF)                                                                               \
    X(64, 4, 1)                                                                                \
    X(64, 16, 1)

template <typename T, int MODE, int CS, int RAD, int BOX>
hipError_t launch_batch_t(const SweepShape& s, const BatchArgs& b, int nblocks, size_t lds,
                          hipStream_t st)
{
#define ABFT_BATCH_CASE(LPR_, NCH_, VEC_)                                                      \
    if (s.lpr == LPR_ && s.nch == NCH_ && s.vec == VEC_) {                                     \
        auto kern = sweep_batch_kernel<T, MODE, CS, LPR_, NCH_, VEC_, RAD, BOX>;               \
        static LdsAllowed lds_ok;                                                              \
        if (hipError_t e = allow_lds(reinterpret_cast<const void*>(kern), lds, lds_ok))        \
            return e;                                                                          \
        hipLaunchKernelGGL(kern, dim3(nblocks), dim3(kBatchWaves * 64), lds, st, b);           \
        return hipGetLastError();                                                              \
    }
    ABFT_BATCH_SHAPES(ABFT_BATCH_CASE)
#undef ABFT_BATCH_CASE
    return hipErrorInvalidValue;
}

template <typename T, int MODE, int CS, int RAD, int BOX>
int occupancy_t(const SweepShape& s, size_t lds)
{
    int n = 0;
#define ABFT_OCC_CASE(LPR_, NCH_, VEC_)                                                        \
    if (s.lpr == LPR_ && s.nch == NCH_ && s.vec == VEC_) {                                     \
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(                                      \
                &n, sweep_batch_kernel<T, MODE, CS, LPR_, NCH_, VEC_, RAD, BOX>,               \
                kBatchWaves * 64, lds) != hipSuccess)                                          \
            n = 1;                                                                             \
        return n > 0 ? n : 1;                                                                  \
    }
    ABFT_BATCH_SHAPES(ABFT_OCC_CASE)
#undef ABFT_OCC_CASE
    return 1;
}
#undef ABFT_BATCH_SHAPES

// Launch and occupancy for one stencil form (radius 1 or 2 star, box) and one dtype, every
// mode and checksum accumulation; each (form, dtype) pair is instantiated in a translation
// unit of its own (ABFT_BATCH_TU), so that they compile in parallel.
template <typename T, int RAD, int BOX>
hipError_t launch_batch_dt(int mode, int csum, const SweepShape& s, const BatchArgs& b,
                           int nblocks, size_t lds, hipStream_t st)
{
    if (mode == MODE_PLAIN)
        return launch_batch_t<T, MODE_PLAIN, CS_F64, RAD, BOX>(s, b, nblocks, lds, st);
    if constexpr (sizeof(T) == 4) {
        if (csum == CS_F32C) {
            if (mode == MODE_PROTM)
                return launch_batch_t<T, MODE_PROTM, CS_F32C, RAD, BOX>(s, b, nblocks, lds, st);
            return launch_batch_t<T, MODE_PROT, CS_F32C, RAD, BOX>(s, b, nblocks, lds, st);
        }
    }
    if (mode == MODE_PROTM)
        return launch_batch_t<T, MODE_PROTM, CS_F64, RAD, BOX>(s, b, nblocks, lds, st);
    return launch_batch_t<T, MODE_PROT, CS_F64, RAD, BOX>(s, b, nblocks, lds, st);
}

template <typename T, int RAD, int BOX>
int occupancy_dt(int mode, int csum, const SweepShape& s, size_t lds)
{
    if (mode == MODE_PLAIN) return occupancy_t<T, MODE_PLAIN, CS_F64, RAD, BOX>(s, lds);
    if constexpr (sizeof(T) == 4) {
        if (csum == CS_F32C) {
            if (mode == MODE_PROTM) return occupancy_t<T, MODE_PROTM, CS_F32C, RAD, BOX>(s, lds);
            return occupancy_t<T, MODE_PROT, CS_F32C, RAD, BOX>(s, lds);
        }
    }
    if (mode == MODE_PROTM) return occupancy_t<T, MODE_PROTM, CS_F64, RAD, BOX>(s, lds);
    return occupancy_t<T, MODE_PROT, CS_F64, RAD, BOX>(s, lds);
}

#define ABFT_BATCH_TU(NAME, T, RAD, BOX)                                                       \
    hipError_t launch_batch_##NAME(int mode, int csum, const SweepShape& s, const BatchArgs& b, \
                                   int nblocks, size_t lds, hipStream_t st)                    \
    {                                                                                          \
        return launch_batch_dt<T, RAD, BOX>(mode, csum, s, b, nblocks, lds, st);               \
    }                                                                                          \
    int batch_occupancy_##NAME(int mode, int csum, const SweepShape& s, size_t lds)            \
    {                                                                                          \
        return occupancy_dt<T, RAD, BOX>(mode, csum, s, lds);                                  \
    }

// Launches holding several chunk counts (radius-1 stars, 16-byte accesses): 16 or 64 lanes
// per row, chunk counts (4, 2, 1), (4, 2), (4, 1), (2, 1).
#define ABFT_BATCH_MULTI(X)                                                                    \
    X(16, 4, 2, 1)                                                                             \
    X(16, 4, 2, 0)                                                                             \
    X(16, 4, 1, 0)                                                                             \
    X(16, 2, 1, 0)                                                                             \
    X(64, 4, 2, 1)                                                                             \
    X(64, 4, 2, 0)                                                                             \
    X(64, 4, 1, 0)                                                                             \
    X(64, 2, 1, 0)

template <typename T, int MODE, int CS>
hipError_t launch_batch_multi_t(const SweepShape& s, const BatchArgs& b, int nblocks, size_t lds,
                                hipStream_t st)
{
    constexpr int VF = 16 / (int)sizeof(T);
#define ABFT_MULTI_CASE(LPR_, A_, B_, C_)                                                      \
    if (s.lpr == LPR_ && s.nch == A_ && s.nchb == B_ && s.nchc == C_ && s.vec == VF) {         \
        auto kern = sweep_batch_kernel<T, MODE, CS, LPR_, A_, VF, 1, 0, B_, C_>;               \
        static LdsAllowed lds_ok;                                                              \
        if (hipError_t e = allow_lds(reinterpret_cast<const void*>(kern), lds, lds_ok))        \
            return e;                                                                          \
        hipLaunchKernelGGL(kern, dim3(nblocks), dim3(kBatchWaves * 64), lds, st, b);           \
        return hipGetLastError();                                                              \
    }
    ABFT_BATCH_MULTI(ABFT_MULTI_CASE)
#undef ABFT_MULTI_CASE
    return hipErrorInvalidValue;
}

template <typename T, int MODE, int CS>
int occupancy_multi_t(const SweepShape& s, size_t lds)
{
    constexpr int VF = 16 / (int)sizeof(T);
    int n = 0;
#define ABFT_MULTI_OCC(LPR_, A_, B_, C_)                                                       \
    if (s.lpr == LPR_ && s.nch == A_ && s.nchb == B_ && s.nchc == C_ && s.vec == VF) {         \
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(                                      \
                &n, sweep_batch_kernel<T, MODE, CS, LPR_, A_, VF, 1, 0, B_, C_>,               \
                kBatchWaves * 64, lds) != hipSuccess)                                          \
            n = 1;                                                                             \
        return n > 0 ? n : 1;                                                                  \
    }
    ABFT_BATCH_MULTI(ABFT_MULTI_OCC)
#undef ABFT_MULTI_OCC
    return 1;
}
#undef ABFT_BATCH_MULTI

template <typename T>
hipError_t launch_batch_multi_dt(int mode, int csum, const SweepShape& s, const BatchArgs& b,
                                 int nblocks, size_t lds, hipStream_t st)
{
    if (mode == MODE_PLAIN) return launch_batch_multi_t<T, MODE_PLAIN, CS_F64>(s, b, nblocks, lds, st);
    if constexpr (sizeof(T) == 4) {
        if (csum == CS_F32C) {
            if (mode == MODE_PROTM)
                return launch_batch_multi_t<T, MODE_PROTM, CS_F32C>(s, b, nblocks, lds, st);
            return launch_batch_multi_t<T, MODE_PROT, CS_F32C>(s, b, nblocks, lds, st);
        }
    }
    if (mode == MODE_PROTM) return launch_batch_multi_t<T, MODE_PROTM, CS_F64>(s, b, nblocks, lds, st);
    return launch_batch_multi_t<T, MODE_PROT, CS_F64>(s, b, nblocks, lds, st);
}

template <typename T>
int occupancy_multi_dt(int mode, int csum, const SweepShape& s, size_t lds)
{
    if (mode == MODE_PLAIN) return occupancy_multi_t<T, MODE_PLAIN, CS_F64>(s, lds);
    if constexpr (sizeof(T) == 4) {
        if (csum == CS_F32C) {
            if (mode == MODE_PROTM) return occupancy_multi_t<T, MODE_PROTM, CS_F32C>(s, lds);
            return occupancy_multi_t<T, MODE_PROT, CS_F32C>(s, lds);
        }
    }
    if (mode == MODE_PROTM) return occupancy_multi_t<T, MODE_PROTM, CS_F64>(s, lds);
    return occupancy_multi_t<T, MODE_PROT, CS_F64>(s, lds);
}

#define ABFT_BATCH_MULTI_TU(NAME, T)                                                           \
    hipError_t launch_batch_##NAME(int mode, int csum, const SweepShape& s, const BatchArgs& b, \
                                   int nblocks, size_t lds, hipStream_t st)                    \
    {                                                                                          \
        return launch_batch_multi_dt<T>(mode, csum, s, b, nblocks, lds, st);                   \
    }                                                                                          \
    int batch_occupancy_##NAME(int mode, int csum, const SweepShape& s, size_t lds)            \
    {                                                                                          \
        return occupancy_multi_dt<T>(mode, csum, s, lds);                                      \
    }

}  // namespace abft
