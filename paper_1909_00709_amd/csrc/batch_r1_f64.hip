// Instantiations of the batched sweep for radius-1 stars, f64 grids.
#include "abft_batch.h"

namespace abft {

ABFT_BATCH_TU(r1_f64, double, 1, 0)

}  // namespace abft
