// Instantiations of the batched sweep for radius-1 stars, f32 grids, in launches that hold
// grids of two or three chunk counts.
#include "abft_batch.h"

namespace abft {

ABFT_BATCH_MULTI_TU(r1x_f32, float)

}  // namespace abft
