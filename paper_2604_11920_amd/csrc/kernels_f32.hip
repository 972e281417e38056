// FP32-vector instantiations: the FP32 solver and the inner solves of the
// BF16/FP16 forms.
#include "lsqr_kernels.cuh"

namespace lsqr {
LSQR_INSTANTIATE_LAUNCHERS(float)
}  // namespace lsqr
