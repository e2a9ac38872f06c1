// Fused batched forward kernels (generation 2) for tap counts 2, 4, 6, 8.
#include "batch_kernels.hpp"

namespace lr {
LR_INSTANTIATE_BATCH_FWD(2, 2)
LR_INSTANTIATE_BATCH_FWD(4, 2)
LR_INSTANTIATE_BATCH_FWD(6, 2)
LR_INSTANTIATE_BATCH_FWD(8, 2)
}  // namespace lr
