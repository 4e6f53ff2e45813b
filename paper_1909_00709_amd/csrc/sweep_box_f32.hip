// Instantiations of the 27-point box sweep: float grids, all variants.
#include "abft_box.h"

namespace abft {

hipError_t launch_sweep_box_f32(int mode, int csum, const SweepShape& s, const SweepArgs& a,
                                hipStream_t st, size_t lds)
{
    if (mode == MODE_PLAIN) return launch_sweep_box_t<float, MODE_PLAIN, CS_F64>(s, a, st, lds);
    if (mode == MODE_CSUM) {
        if (csum == CS_F32C) return launch_sweep_box_t<float, MODE_CSUM, CS_F32C>(s, a, st, lds);
        return launch_sweep_box_t<float, MODE_CSUM, CS_F64>(s, a, st, lds);
    }
    if (csum == CS_F32C) return launch_sweep_box_t<float, MODE_PROT, CS_F32C>(s, a, st, lds);
    return launch_sweep_box_t<float, MODE_PROT, CS_F64>(s, a, st, lds);
}

}  // namespace abft
