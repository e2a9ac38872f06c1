// Adjoint kernels instantiated for tap counts 10, 12, 14, 16.
#include "adjoint_kernels.hpp"

namespace lr {
LR_INSTANTIATE_ADJOINT(10)
LR_INSTANTIATE_ADJOINT(12)
LR_INSTANTIATE_ADJOINT(14)
LR_INSTANTIATE_ADJOINT(16)
}  // namespace lr
