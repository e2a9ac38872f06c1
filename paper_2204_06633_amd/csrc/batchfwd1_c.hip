// Fused batched forward kernels (generation 1) for tap counts 18, 20, 22, 24.
#include "batch_kernels.hpp"

namespace lr {
LR_INSTANTIATE_BATCH_FWD(18, 1)
LR_INSTANTIATE_BATCH_FWD(20, 1)
LR_INSTANTIATE_BATCH_FWD(22, 1)
LR_INSTANTIATE_BATCH_FWD(24, 1)
}  // namespace lr
