// Conjugate-gradient kernels instantiated for the all-FP64 path.
#include "cg_launch.h"

namespace bem {
BEM_INSTANTIATE_CG(double)
}
