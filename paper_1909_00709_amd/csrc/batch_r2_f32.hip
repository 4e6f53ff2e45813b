// Instantiations of the batched sweep for radius-2 stars, f32 grids.
#include "abft_batch.h"

namespace abft {

ABFT_BATCH_TU(r2_f32, float, 2, 0)

}  // namespace abft
