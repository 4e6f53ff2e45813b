// Instantiations of the sweep kernel for radius-2 stars: float grid, plain and row-checksum
// variants.
#include "abft_sweep.h"

namespace abft {

hipError_t launch_sweep_r2_f32_pc(int mode, int csum, const SweepShape& s, const SweepArgs& a,
                                  hipStream_t st, size_t lds)
{
    if (mode == MODE_PLAIN) return launch_sweep_t<float, MODE_PLAIN, CS_F64, 2>(s, a, st, lds);
    if (mode != MODE_CSUM) return hipErrorInvalidValue;
    if (csum == CS_F32C) return launch_sweep_t<float, MODE_CSUM, CS_F32C, 2>(s, a, st, lds);
    return launch_sweep_t<float, MODE_CSUM, CS_F64, 2>(s, a, st, lds);
}

}  // namespace abft
