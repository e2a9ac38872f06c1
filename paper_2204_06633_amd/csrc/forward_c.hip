// Forward kernels instantiated for tap counts 18, 20, 22, 24.
#include "forward_kernels.hpp"

namespace lr {
LR_INSTANTIATE_FORWARD(18)
LR_INSTANTIATE_FORWARD(20)
LR_INSTANTIATE_FORWARD(22)
LR_INSTANTIATE_FORWARD(24)
}  // namespace lr
