// Instantiations of the batched sweep for 27-point box stencils.
#include "abft_batch.h"

namespace abft {

hipError_t launch_batch_box(int dtype, int mode, int csum, const SweepShape& s,
                             const BatchArgs& b, int nblocks, size_t lds, hipStream_t st)
{
    return launch_batch_form<1, 1>(dtype, mode, csum, s, b, nblocks, lds, st);
}

int batch_occupancy_box(int dtype, int mode, int csum, const SweepShape& s, size_t lds)
{
    return occupancy_form<1, 1>(dtype, mode, csum, s, lds);
}

}  // namespace abft
