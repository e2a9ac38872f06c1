// Forward kernels instantiated for tap counts 26, 28, 30, 32.
#include "forward_kernels.hpp"

namespace lr {
LR_INSTANTIATE_FORWARD(26)
LR_INSTANTIATE_FORWARD(28)
LR_INSTANTIATE_FORWARD(30)
LR_INSTANTIATE_FORWARD(32)
}  // namespace lr
