// Instantiations of the offline rollback recompute for 27-point box stencils: double grids.
#include "abft_recover.h"

namespace abft {

hipError_t launch_recover_box_f64(int csum, const SweepShape& s, const RecoverArgs& r,
                                  size_t lds, int num_cus, hipStream_t st)
{
    (void)csum;
    return launch_recover_t<double, CS_F64, 1, 1>(s, r, lds, num_cus, st);
}

}  // namespace abft
