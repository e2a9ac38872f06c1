// Adjoint kernels instantiated for tap counts 26, 28, 30, 32.
#include "adjoint_kernels.hpp"

namespace lr {
LR_INSTANTIATE_ADJOINT(26)
LR_INSTANTIATE_ADJOINT(28)
LR_INSTANTIATE_ADJOINT(30)
LR_INSTANTIATE_ADJOINT(32)
}  // namespace lr
