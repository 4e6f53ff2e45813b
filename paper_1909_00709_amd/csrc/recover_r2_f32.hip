// Instantiations of the offline rollback recompute for radius-2 stars: float grids.
#include "abft_recover.h"

namespace abft {

hipError_t launch_recover_r2_f32(int csum, const SweepShape& s, const RecoverArgs& r, size_t lds,
                                 int num_cus, hipStream_t st)
{
    if (csum == CS_F32C) return launch_recover_t<float, CS_F32C, 2>(s, r, lds, num_cus, st);
    return launch_recover_t<float, CS_F64, 2>(s, r, lds, num_cus, st);
}

}  // namespace abft
