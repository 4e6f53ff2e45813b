// Rollback recompute of an offline window (Section 4) in one launch.
//
// When the window check flags a mismatch, the window's k sweeps are run again from the
// checkpoint, the fault plan taken as attempt 1.  Launching them as k kernels would leave k
// guarded launches in every window, each dispatching a full grid of blocks that exits at once
// when nothing was flagged.  Here one launch holds at most one wave of blocks (occupancy x
// compute units, so that all of them are resident together once the stream's previous kernel
// has finished); each block takes tiles of a sweep in turn, and a grid barrier separates the
// sweeps.  The last sweep also forms the direct row checksums, which the following guarded
// check compares with the window's interpolation.  (A cooperative launch would guarantee the
// residency, but on this runtime it idles the device for about 11 us on each side of the
// launch, more than the guarded launches it replaces.)  If other streams hold compute units,
// late blocks start when those are released.  Every barrier wait is bounded: a block that has
// waited about three seconds gives up, counts the timeout and leaves, so the grid always
// drains, and the next check reports the failure.
#pragma once

#include "abft_box.h"

namespace abft {

// Grid-wide barrier over a counter that only grows during a launch: round r waits until
// r * gridDim.x blocks have arrived.  Thread 0 publishes the block's writes (agent-scope
// release) before arriving and acquires after the wait.  Returns false on a timeout.
__device__ __forceinline__ bool grid_barrier(uint32_t* bar, unsigned target,
                                             unsigned long long* timeouts)
{
    __shared__ int ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        atomicAdd(bar, 1u);
        int good = 1;
        unsigned spins = 0;
        while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > kBarrierSpinLimit) {
                good = 0;
                atomicAdd(timeouts, 1ull);
                break;
            }
        }
        __threadfence();
        ok = good;
    }
    __syncthreads();
    return ok != 0;
}

template <typename T, int CS, int LPR, int NCH, int VEC, int NW, int RAD, int BOX>
__global__ void __launch_bounds__(NW * 64) recover_kernel(const RecoverArgs r)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    if (r.guard != nullptr && *r.guard == 0u) return;
    Counters* cnt = r.a.cnt;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        atomicAdd(&cnt->rollbacks, 1ull);
        emit_event(cnt, r.a.ev, r.a.ev_cap, r.t_first, ABFT_EV_ROLLBACK, -1, -1, r.k, 0.0, 0.0,
                   0);
    }
    const unsigned nb = gridDim.x;
    for (int j = 0; j < r.k; ++j) {
        SweepArgs a = r.a;
        a.uin = j == 0 ? r.ckpt : ((j & 1) ? r.odd : r.even);
        a.uout = const_cast<void*>((j & 1) ? r.even : r.odd);
        a.t_off = r.t_first + j;
        a.E = r.E != nullptr ? r.E + (size_t)j * a.nz * a.ny : nullptr;
        for (int tile = blockIdx.x; tile < a.ntiles; tile += (int)nb) {
            if constexpr (BOX) {
                if (j == r.k - 1)
                    sweep_box_tile<T, MODE_CSUM, CS, LPR, NCH, VEC, NW>(a, tile, smem_raw);
                else
                    sweep_box_tile<T, MODE_PLAIN, CS, LPR, NCH, VEC, NW>(a, tile, smem_raw);
            } else {
                if (j == r.k - 1)
                    sweep_tile<T, MODE_CSUM, CS, LPR, NCH, VEC, 1, NW, RAD>(a, tile, smem_raw);
                else
                    sweep_tile<T, MODE_PLAIN, CS, LPR, NCH, VEC, 1, NW, RAD>(a, tile, smem_raw);
            }
            __syncthreads();  // the tile's LDS use is over
        }
        if (j + 1 < r.k && !grid_barrier(r.bar, (unsigned)(j + 1) * nb, &cnt->barrier_timeouts))
            return;
    }
    // the last block to leave rewinds the barrier for the next launch
    if (threadIdx.x == 0 && atomicAdd(&r.bar[1], 1u) == nb - 1) {
        atomicExch(&r.bar[0], 0u);
        atomicExch(&r.bar[1], 0u);
    }
}

template <typename T, int CS, int RAD, int BOX = 0>
hipError_t launch_recover_t(const SweepShape& s, const RecoverArgs& r, size_t lds, int num_cus,
                            hipStream_t st)
{
#define ABFT_RECOVER_CASE_NW(LPR_, NCH_, VEC_, NW_)                                            \
    if (s.lpr == LPR_ && s.nch == NCH_ && s.vec == VEC_ && s.nw == NW_) {                      \
        auto kern = recover_kernel<T, CS, LPR_, NCH_, VEC_, NW_, RAD, BOX>;                    \
        static LdsAllowed lds_ok;                                                              \
        static size_t occ_lds = 0;                                                             \
        static int occ = 0;                                                                    \
        if (hipError_t e = allow_lds(reinterpret_cast<const void*>(kern), lds, lds_ok))        \
            return e;                                                                          \
        if (occ_lds != lds || occ < 1) {                                                       \
            hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, NW_ * 64,  \
                                                                        lds);                  \
            if (e != hipSuccess) return e;                                                     \
            if (occ < 1) return hipErrorInvalidConfiguration;                                  \
            occ_lds = lds;                                                                     \
        }                                                                                      \
        const int64_t most = (int64_t)occ * num_cus;                                           \
        const int nb = (int)(r.a.ntiles < most ? r.a.ntiles : most);                           \
        hipLaunchKernelGGL(kern, dim3(nb), dim3(NW_ * 64), lds, st, r);                        \
        return hipGetLastError();                                                              \
    }
#define ABFT_RECOVER_CASE(LPR_, NCH_, VEC_)                                                    \
    ABFT_RECOVER_CASE_NW(LPR_, NCH_, VEC_, 4)                                                  \
    if constexpr (NCH_ * VEC_ * sizeof(T) <= kWideBlockLaneBytes) {                            \
        ABFT_RECOVER_CASE_NW(LPR_, NCH_, VEC_, 8)                                              \
    }
    constexpr int VF = 16 / (int)sizeof(T);
    ABFT_RECOVER_CASE(16, 1, VF)
    ABFT_RECOVER_CASE(16, 2, VF)
    ABFT_RECOVER_CASE(16, 4, VF)
    ABFT_RECOVER_CASE(64, 1, VF)
    ABFT_RECOVER_CASE(64, 2, VF)
    ABFT_RECOVER_CASE(64, 4, VF)
    ABFT_RECOVER_CASE(64, 8, VF)
    ABFT_RECOVER_CASE(64, 4, 1)
    ABFT_RECOVER_CASE(64, 16, 1)
#undef ABFT_RECOVER_CASE
#undef ABFT_RECOVER_CASE_NW
    return hipErrorInvalidValue;
}

}  // namespace abft
