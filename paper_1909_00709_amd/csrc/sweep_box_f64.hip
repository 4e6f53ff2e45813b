// Instantiations of the 27-point box sweep: double grids, all variants.
#include "abft_box.h"

namespace abft {

hipError_t launch_sweep_box_f64(int mode, int csum, const SweepShape& s, const SweepArgs& a,
                                hipStream_t st, size_t lds)
{
    (void)csum;
    if (mode == MODE_PLAIN) return launch_sweep_box_t<double, MODE_PLAIN, CS_F64>(s, a, st, lds);
    if (mode == MODE_CSUM) return launch_sweep_box_t<double, MODE_CSUM, CS_F64>(s, a, st, lds);
    return launch_sweep_box_t<double, MODE_PROT, CS_F64>(s, a, st, lds);
}

}  // namespace abft
