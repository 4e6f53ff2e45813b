// Instantiations of the box sweep kernel: float grid, protected variant with the input-side
// check.
#include "abft_box.h"

namespace abft {

hipError_t launch_sweep_box_f32_protm(int csum, const SweepShape& s, const SweepArgs& a,
                                      hipStream_t st, size_t lds)
{
    if (csum == CS_F32C) return launch_sweep_box_t<float, MODE_PROTM, CS_F32C>(s, a, st, lds);
    return launch_sweep_box_t<float, MODE_PROTM, CS_F64>(s, a, st, lds);
}

}  // namespace abft
