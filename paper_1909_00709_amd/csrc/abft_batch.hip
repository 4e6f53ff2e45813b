// Batched sweep: many independent grids of uneven sizes swept by one launch.
//
// The tiles of all grids form one list, largest first.  In the persistent form a fixed grid of
// blocks (enough to fill the compute units once) pops tiles from an atomic counter, fetching
// the next index while the current tile runs; in the direct form block b takes tile b and the
// hardware dispatcher does the balancing (abft_batch.h).  This file holds the shapes, the LDS
// size and the dispatch by stencil form and dtype (instantiated in batch_{r1,r2,box}_{f32,f64}).
#include "abft_internal.h"

namespace abft {

bool batch_shape_supported(int dtype, const SweepShape& s)
{
    const int vf = dtype == ABFT_F32 ? 4 : 2;
    if (s.nw != kBatchWaves || s.pf != 1) return false;
    if (s.nchb > 0) {
        // launches of several chunk counts: radius-1 stars, 16-byte accesses, 16 or 64 lanes,
        // chunk counts (4, 2, 1), (4, 2), (4, 1), (2, 1)
        if (s.rad != 1 || s.box || s.vec != vf || (s.lpr != 16 && s.lpr != 64)) return false;
        if (s.nch == 4)
            return (s.nchb == 2 && (s.nchc == 1 || s.nchc == 0)) || (s.nchb == 1 && s.nchc == 0);
        return s.nch == 2 && s.nchb == 1 && s.nchc == 0;
    }
    if (s.nchc != 0) return false;
    if (s.vec == vf) return (s.lpr == 16 || s.lpr == 64) && (s.nch == 1 || s.nch == 2 || s.nch == 4);
    return s.vec == 1 && s.lpr == 64 && (s.nch == 4 || s.nch == 16);
}

size_t batch_lds_bytes(int dtype, int maxnx, int maxtz, const SweepShape& s, bool input_check)
{
    SweepShape t = s;
    t.tz = maxtz;
    return sweep_lds_bytes(dtype, maxnx, t, input_check);
}

hipError_t launch_sweep_batch(int dtype, int mode, int csum, const SweepShape& s,
                              const BatchArgs& b, int nblocks, size_t lds, hipStream_t st)
{
    if (!batch_shape_supported(dtype, s) || nblocks < 1) return hipErrorInvalidValue;
    const bool f32 = dtype == ABFT_F32;
    if (s.nchb > 0)
        return f32 ? launch_batch_r1x_f32(mode, csum, s, b, nblocks, lds, st)
                   : launch_batch_r1x_f64(mode, csum, s, b, nblocks, lds, st);
    if (s.box)
        return f32 ? launch_batch_box_f32(mode, csum, s, b, nblocks, lds, st)
                   : launch_batch_box_f64(mode, csum, s, b, nblocks, lds, st);
    if (s.rad == 2)
        return f32 ? launch_batch_r2_f32(mode, csum, s, b, nblocks, lds, st)
                   : launch_batch_r2_f64(mode, csum, s, b, nblocks, lds, st);
    return f32 ? launch_batch_r1_f32(mode, csum, s, b, nblocks, lds, st)
               : launch_batch_r1_f64(mode, csum, s, b, nblocks, lds, st);
}

int batch_blocks_per_cu(int dtype, int mode, int csum, const SweepShape& s, size_t lds)
{
    const bool f32 = dtype == ABFT_F32;
    if (s.nchb > 0)
        return f32 ? batch_occupancy_r1x_f32(mode, csum, s, lds)
                   : batch_occupancy_r1x_f64(mode, csum, s, lds);
    if (s.box)
        return f32 ? batch_occupancy_box_f32(mode, csum, s, lds)
                   : batch_occupancy_box_f64(mode, csum, s, lds);
    if (s.rad == 2)
        return f32 ? batch_occupancy_r2_f32(mode, csum, s, lds)
                   : batch_occupancy_r2_f64(mode, csum, s, lds);
    return f32 ? batch_occupancy_r1_f32(mode, csum, s, lds)
               : batch_occupancy_r1_f64(mode, csum, s, lds);
}

}  // namespace abft
