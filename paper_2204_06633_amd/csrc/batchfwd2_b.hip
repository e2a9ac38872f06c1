// Fused batched forward kernels (generation 2) for tap counts 10, 12, 14, 16.
#include "batch_kernels.hpp"

namespace lr {
LR_INSTANTIATE_BATCH_FWD(10, 2)
LR_INSTANTIATE_BATCH_FWD(12, 2)
LR_INSTANTIATE_BATCH_FWD(14, 2)
LR_INSTANTIATE_BATCH_FWD(16, 2)
}  // namespace lr
