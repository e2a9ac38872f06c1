// Batched adjoint kernels for tap counts 10, 12, 14, 16.
#include "batch_adjoint_kernels.hpp"

namespace lr {
LR_INSTANTIATE_BATCH_ADJ(10)
LR_INSTANTIATE_BATCH_ADJ(12)
LR_INSTANTIATE_BATCH_ADJ(14)
LR_INSTANTIATE_BATCH_ADJ(16)
}  // namespace lr
