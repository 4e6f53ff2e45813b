// Instantiations of the radius-2 sweep kernel: float grid, protected variant with the
// input-side check.
#include "abft_sweep.h"

namespace abft {

hipError_t launch_sweep_r2_f32_protm(int csum, const SweepShape& s, const SweepArgs& a,
                                     hipStream_t st, size_t lds)
{
    if (csum == CS_F32C) return launch_sweep_t<float, MODE_PROTM, CS_F32C, 2>(s, a, st, lds);
    return launch_sweep_t<float, MODE_PROTM, CS_F64, 2>(s, a, st, lds);
}

}  // namespace abft
