// Forward kernels instantiated for tap counts 2, 4, 6, 8.
#include "forward_kernels.hpp"

namespace lr {
LR_INSTANTIATE_FORWARD(2)
LR_INSTANTIATE_FORWARD(4)
LR_INSTANTIATE_FORWARD(6)
LR_INSTANTIATE_FORWARD(8)
}  // namespace lr
