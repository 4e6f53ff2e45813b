// Instantiations of the batched sweep for radius-1 stars, f32 grids.
#include "abft_batch.h"

namespace abft {

ABFT_BATCH_TU(r1_f32, float, 1, 0)

}  // namespace abft
