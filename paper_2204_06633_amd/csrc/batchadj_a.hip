// Batched adjoint kernels for tap counts 2, 4, 6, 8.
#include "batch_adjoint_kernels.hpp"

namespace lr {
LR_INSTANTIATE_BATCH_ADJ(2)
LR_INSTANTIATE_BATCH_ADJ(4)
LR_INSTANTIATE_BATCH_ADJ(6)
LR_INSTANTIATE_BATCH_ADJ(8)
}  // namespace lr
