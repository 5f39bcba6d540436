// Batched CG iteration kernels (double instantiation).
#include "batch.h"

namespace bem {
template hipError_t launch_batch_iterations<double>(const Geom&, const SpecView<double>&,
                                                  const BatchSlot<double>*, int, unsigned, int,
                                                  hipStream_t);
}  // namespace bem
