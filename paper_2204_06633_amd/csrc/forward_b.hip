// Forward kernels instantiated for tap counts 10, 12, 14, 16.
#include "forward_kernels.hpp"

namespace lr {
LR_INSTANTIATE_FORWARD(10)
LR_INSTANTIATE_FORWARD(12)
LR_INSTANTIATE_FORWARD(14)
LR_INSTANTIATE_FORWARD(16)
}  // namespace lr
