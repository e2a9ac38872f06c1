// Fused batched forward kernels (generation 1) for tap counts 26, 28, 30, 32.
#include "batch_kernels.hpp"

namespace lr {
LR_INSTANTIATE_BATCH_FWD(26, 1)
LR_INSTANTIATE_BATCH_FWD(28, 1)
LR_INSTANTIATE_BATCH_FWD(30, 1)
LR_INSTANTIATE_BATCH_FWD(32, 1)
}  // namespace lr
