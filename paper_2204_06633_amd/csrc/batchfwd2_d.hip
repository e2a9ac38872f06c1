// Fused batched forward kernels (generation 2) for tap counts 26, 28, 30, 32.
#include "batch_kernels.hpp"

namespace lr {
LR_INSTANTIATE_BATCH_FWD(26, 2)
LR_INSTANTIATE_BATCH_FWD(28, 2)
LR_INSTANTIATE_BATCH_FWD(30, 2)
LR_INSTANTIATE_BATCH_FWD(32, 2)
}  // namespace lr
