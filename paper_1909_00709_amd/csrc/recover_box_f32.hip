// Instantiations of the offline rollback recompute for 27-point box stencils: float grids.
#include "abft_recover.h"

namespace abft {

hipError_t launch_recover_box_f32(int csum, const SweepShape& s, const RecoverArgs& r,
                                  size_t lds, int num_cus, hipStream_t st)
{
    if (csum == CS_F32C) return launch_recover_t<float, CS_F32C, 1, 1>(s, r, lds, num_cus, st);
    return launch_recover_t<float, CS_F64, 1, 1>(s, r, lds, num_cus, st);
}

}  // namespace abft
