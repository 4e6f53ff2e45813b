// Instantiations of the batched sweep for radius-1 stars, f64 grids, in launches that hold
// grids of two or three chunk counts.
#include "abft_batch.h"

namespace abft {

ABFT_BATCH_MULTI_TU(r1x_f64, double)

}  // namespace abft
