// The batched sweep kernel: many independent grids of uneven sizes swept by one launch.
//
// The tiles of all grids form one list, largest first.  In the persistent form a fixed grid of
// blocks (enough to fill the compute units once) pops tiles from an atomic counter, fetching
// the next index while the current tile runs; in the direct form block b takes tile b and the
// hardware dispatcher does the balancing.  Every tile runs the same fused sweep/checksum code
// as a single grid (sweep_tile, or sweep_box_tile for box stencils), with that grid's
// descriptor; all grids of a batch share the stencil form (radius and box), each has its own
// weights.
#pragma once

#include "abft_box.h"

namespace abft {

template <typename T, int MODE, int CS, int LPR, int NCH, int VEC, int RAD, int BOX>
__global__ void __launch_bounds__(kSweepBlock) sweep_batch_kernel(const BatchArgs b)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    __shared__ int sh_next;
    const int p = b.parity;
    if (blockIdx.x == 0) {
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
        it = sh_next;
    } else {
        it = blockIdx.x;
    }
    while (it < b.ntiles) {
        __syncthreads();  // everyone has read sh_next; the previous tile's LDS use is over
        if (b.persistent && threadIdx.x == 0) sh_next = (int)atomicAdd(&b.queue[0], 1u);
        const int2 gt = b.order[it];
        const GridDesc& d = b.grids[gt.x];
        SweepArgs a{};
        a.uin = d.u[p];
        a.uout = d.u[p ^ 1];
        a.C = d.C;
        a.c_scalar = d.c_scalar;
        a.st = d.st;
        a.nx = d.nx;
        a.ny = d.ny;
        a.nz = d.nz;
        a.tz = d.tz;
        a.nyb = d.nyb;
        a.ntiles = d.ntiles;
        a.attempt = b.attempt;
        a.t_base = b.t_base;
        a.t_off = b.t_off;
        a.Bt = d.B[p];
        a.Bn = d.B[p ^ 1];
        a.Wn = d.W[p ^ 1];
        a.cB = d.cB;
        a.eps = b.eps;
        a.slot = d.slot[p];
        a.cnt = b.cnt;
        a.ev = b.ev;
        a.ev_cap = b.ev_cap;
        a.grid = gt.x;
        a.faults = b.faults;
        a.fault_first = b.fault_first;
        a.fault_tmax = b.fault_tmax;
        if constexpr (BOX)
            sweep_box_tile<T, MODE, CS, LPR, NCH, VEC, kSweepBlock / 64>(a, gt.y, smem_raw);
        else
            sweep_tile<T, MODE, CS, LPR, NCH, VEC, 1, kSweepBlock / 64, RAD>(a, gt.y, smem_raw);
        if (!b.persistent) break;
        __syncthreads();
        it = sh_next;
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

template <typename T, int MODE, int CS, int RAD, int BOX>
hipError_t launch_batch_t(const SweepShape& s, const BatchArgs& b, int nblocks, size_t lds,
                          hipStream_t st)
{
#define ABFT_BATCH_CASE(LPR_, NCH_, VEC_)                                                      \
    if (s.lpr == LPR_ && s.nch == NCH_ && s.vec == VEC_) {                                     \
        auto kern = sweep_batch_kernel<T, MODE, CS, LPR_, NCH_, VEC_, RAD, BOX>;               \
        static int lds_set = 0;                                                                \
        if (lds > 65536 && (int)lds > lds_set) {                                               \
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),             \
                                               hipFuncAttributeMaxDynamicSharedMemorySize,      \
                                               (int)lds);                                      \
            if (e != hipSuccess) return e;                                                     \
            lds_set = (int)lds;                                                                \
        }                                                                                      \
        hipLaunchKernelGGL(kern, dim3(nblocks), dim3(kSweepBlock), lds, st, b);                \
        return hipGetLastError();                                                              \
    }
    constexpr int VF = 16 / (int)sizeof(T);
    ABFT_BATCH_CASE(16, 4, VF)
    ABFT_BATCH_CASE(64, 4, VF)
    ABFT_BATCH_CASE(64, 16, 1)
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
                &n, sweep_batch_kernel<T, MODE, CS, LPR_, NCH_, VEC_, RAD, BOX>, kSweepBlock,   \
                lds) != hipSuccess)                                                            \
            n = 1;                                                                             \
        return n > 0 ? n : 1;                                                                  \
    }
    constexpr int VF = 16 / (int)sizeof(T);
    ABFT_OCC_CASE(16, 4, VF)
    ABFT_OCC_CASE(64, 4, VF)
    ABFT_OCC_CASE(64, 16, 1)
#undef ABFT_OCC_CASE
    return 1;
}

// Launch and occupancy for one stencil form (radius 1 or 2 star, box), every mode, checksum
// accumulation and dtype; instantiated once per form in its own translation unit.
template <int RAD, int BOX>
hipError_t launch_batch_form(int dtype, int mode, int csum, const SweepShape& s,
                             const BatchArgs& b, int nblocks, size_t lds, hipStream_t st)
{
    if (dtype == ABFT_F32) {
        if (mode == MODE_PLAIN)
            return launch_batch_t<float, MODE_PLAIN, CS_F64, RAD, BOX>(s, b, nblocks, lds, st);
        if (mode == MODE_PROTM) {
            if (csum == CS_F32C)
                return launch_batch_t<float, MODE_PROTM, CS_F32C, RAD, BOX>(s, b, nblocks, lds, st);
            return launch_batch_t<float, MODE_PROTM, CS_F64, RAD, BOX>(s, b, nblocks, lds, st);
        }
        if (csum == CS_F32C)
            return launch_batch_t<float, MODE_PROT, CS_F32C, RAD, BOX>(s, b, nblocks, lds, st);
        return launch_batch_t<float, MODE_PROT, CS_F64, RAD, BOX>(s, b, nblocks, lds, st);
    }
    if (mode == MODE_PLAIN)
        return launch_batch_t<double, MODE_PLAIN, CS_F64, RAD, BOX>(s, b, nblocks, lds, st);
    if (mode == MODE_PROTM)
        return launch_batch_t<double, MODE_PROTM, CS_F64, RAD, BOX>(s, b, nblocks, lds, st);
    return launch_batch_t<double, MODE_PROT, CS_F64, RAD, BOX>(s, b, nblocks, lds, st);
}

template <int RAD, int BOX>
int occupancy_form(int dtype, int mode, int csum, const SweepShape& s, size_t lds)
{
    if (dtype == ABFT_F32) {
        if (mode == MODE_PLAIN) return occupancy_t<float, MODE_PLAIN, CS_F64, RAD, BOX>(s, lds);
        if (mode == MODE_PROTM) {
            if (csum == CS_F32C) return occupancy_t<float, MODE_PROTM, CS_F32C, RAD, BOX>(s, lds);
            return occupancy_t<float, MODE_PROTM, CS_F64, RAD, BOX>(s, lds);
        }
        if (csum == CS_F32C) return occupancy_t<float, MODE_PROT, CS_F32C, RAD, BOX>(s, lds);
        return occupancy_t<float, MODE_PROT, CS_F64, RAD, BOX>(s, lds);
    }
    if (mode == MODE_PLAIN) return occupancy_t<double, MODE_PLAIN, CS_F64, RAD, BOX>(s, lds);
    if (mode == MODE_PROTM) return occupancy_t<double, MODE_PROTM, CS_F64, RAD, BOX>(s, lds);
    return occupancy_t<double, MODE_PROT, CS_F64, RAD, BOX>(s, lds);
}

}  // namespace abft
