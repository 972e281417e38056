// FP64-vector instantiations: the plain FP64 solver and the FP64 products of
// the mixed-precision refinement.
#include "lsqr_kernels.cuh"

namespace lsqr {
LSQR_INSTANTIATE_LAUNCHERS(double)
}  // namespace lsqr
