// Conjugate-gradient kernels instantiated for the MIXED path (FP32 vectors
// and transforms, FP64 reductions).
#include "cg_launch.h"

namespace bem {
BEM_INSTANTIATE_CG(float)
}
