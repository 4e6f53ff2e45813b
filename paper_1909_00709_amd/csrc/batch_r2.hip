// Instantiations of the batched sweep for radius-2 star stencils.
#include "abft_batch.h"

namespace abft {

hipError_t launch_batch_r2(int dtype, int mode, int csum, const SweepShape& s,
                             const BatchArgs& b, int nblocks, size_t lds, hipStream_t st)
{
    return launch_batch_form<2, 0>(dtype, mode, csum, s, b, nblocks, lds, st);
}

int batch_occupancy_r2(int dtype, int mode, int csum, const SweepShape& s, size_t lds)
{
    return occupancy_form<2, 0>(dtype, mode, csum, s, lds);
}

}  // namespace abft
