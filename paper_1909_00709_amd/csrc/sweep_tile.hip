// Instantiations of the star sweep kernel with tile-local checksums (radius 1 and 2, float and
// double grids).
#include "abft_sweep.h"

namespace abft {

hipError_t launch_sweep_f32_tile(int csum, const SweepShape& s, const SweepArgs& a,
                                 hipStream_t st, size_t lds)
{
    (void)csum;
    if (s.rad == 2) return launch_sweep_t<float, MODE_TILE, CS_F64, 2>(s, a, st, lds);
    return launch_sweep_t<float, MODE_TILE, CS_F64, 1>(s, a, st, lds);
}

hipError_t launch_sweep_f64_tile(int csum, const SweepShape& s, const SweepArgs& a,
                                 hipStream_t st, size_t lds)
{
    (void)csum;
    if (s.rad == 2) return launch_sweep_t<double, MODE_TILE, CS_F64, 2>(s, a, st, lds);
    return launch_sweep_t<double, MODE_TILE, CS_F64, 1>(s, a, st, lds);
}

}  // namespace abft
