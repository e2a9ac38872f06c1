// Fused batched forward kernels (generation 1) for tap counts 2, 4, 6, 8.
#include "batch_kernels.hpp"

namespace lr {
LR_INSTANTIATE_BATCH_FWD(2, 1)
LR_INSTANTIATE_BATCH_FWD(4, 1)
LR_INSTANTIATE_BATCH_FWD(6, 1)
LR_INSTANTIATE_BATCH_FWD(8, 1)
}  // namespace lr
