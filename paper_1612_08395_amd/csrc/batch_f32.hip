// Batched CG iteration kernels (float instantiation).
#include "batch.h"

namespace bem {
template hipError_t launch_batch_iterations<float>(const Geom&, const SpecView<float>&,
                                                  const BatchSlot<float>*, int, unsigned, int,
                                                  hipStream_t);
}  // namespace bem
