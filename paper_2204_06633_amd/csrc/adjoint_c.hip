// Adjoint kernels instantiated for tap counts 18, 20, 22, 24.
#include "adjoint_kernels.hpp"

namespace lr {
LR_INSTANTIATE_ADJOINT(18)
LR_INSTANTIATE_ADJOINT(20)
LR_INSTANTIATE_ADJOINT(22)
LR_INSTANTIATE_ADJOINT(24)
}  // namespace lr
