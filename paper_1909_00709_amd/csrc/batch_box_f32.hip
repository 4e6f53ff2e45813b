// Instantiations of the batched sweep for 27-point box stencils, f32 grids.
#include "abft_batch.h"

namespace abft {

ABFT_BATCH_TU(box_f32, float, 1, 1)

}  // namespace abft
