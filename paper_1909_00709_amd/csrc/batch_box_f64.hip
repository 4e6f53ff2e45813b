// Instantiations of the batched sweep for 27-point box stencils, f64 grids.
#include "abft_batch.h"

namespace abft {

ABFT_BATCH_TU(box_f64, double, 1, 1)

}  // namespace abft
