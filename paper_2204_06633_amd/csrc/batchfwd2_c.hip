// Fused batched forward kernels (generation 2) for tap counts 18, 20, 22, 24.
#include "batch_kernels.hpp"

namespace lr {
LR_INSTANTIATE_BATCH_FWD(18, 2)
LR_INSTANTIATE_BATCH_FWD(20, 2)
LR_INSTANTIATE_BATCH_FWD(22, 2)
LR_INSTANTIATE_BATCH_FWD(24, 2)
}  // namespace lr
