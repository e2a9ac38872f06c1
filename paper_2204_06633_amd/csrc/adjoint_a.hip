// Adjoint kernels instantiated for tap counts 2, 4, 6, 8.
#include "adjoint_kernels.hpp"

namespace lr {
LR_INSTANTIATE_ADJOINT(2)
LR_INSTANTIATE_ADJOINT(4)
LR_INSTANTIATE_ADJOINT(6)
LR_INSTANTIATE_ADJOINT(8)
}  // namespace lr
