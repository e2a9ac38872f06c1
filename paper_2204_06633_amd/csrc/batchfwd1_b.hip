// Fused batched forward kernels (generation 1) for tap counts 10, 12, 14, 16.
#include "batch_kernels.hpp"

namespace lr {
LR_INSTANTIATE_BATCH_FWD(10, 1)
LR_INSTANTIATE_BATCH_FWD(12, 1)
LR_INSTANTIATE_BATCH_FWD(14, 1)
LR_INSTANTIATE_BATCH_FWD(16, 1)
}  // namespace lr
