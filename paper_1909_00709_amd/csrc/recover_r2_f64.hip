// Instantiations of the offline rollback recompute for radius-2 stars: double grids.
#include "abft_recover.h"

namespace abft {

hipError_t launch_recover_r2_f64(int csum, const SweepShape& s, const RecoverArgs& r, size_t lds,
                                 int num_cus, hipStream_t st)
{
    (void)csum;
    return launch_recover_t<double, CS_F64, 2>(s, r, lds, num_cus, st);
}

}  // namespace abft
