// Instantiations of the radius-2 sweep kernel: double grid, protected variant with the
// input-side check.
#include "abft_sweep.h"

namespace abft {

hipError_t launch_sweep_r2_f64_protm(int csum, const SweepShape& s, const SweepArgs& a,
                                     hipStream_t st, size_t lds)
{
    (void)csum;
    return launch_sweep_t<double, MODE_PROTM, CS_F64, 2>(s, a, st, lds);
}

}  // namespace abft
