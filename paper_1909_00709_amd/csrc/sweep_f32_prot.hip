// Instantiations of the sweep kernel: float grid, prot variant.
#include "abft_sweep.h"

namespace abft {

hipError_t launch_sweep_f32_prot(int csum, const SweepShape& s, const SweepArgs& a, hipStream_t st,
                              size_t lds)
{
    (void)csum;
    if (csum == CS_F64) return launch_sweep_t<float, MODE_PROT, CS_F64, 1>(s, a, st, lds);
    if (csum == CS_F32C) return launch_sweep_t<float, MODE_PROT, CS_F32C, 1>(s, a, st, lds);
    return hipErrorInvalidValue;
}

}  // namespace abft
