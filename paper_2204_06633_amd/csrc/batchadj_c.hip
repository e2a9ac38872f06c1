// Batched adjoint kernels for tap counts 18, 20, 22, 24.
#include "batch_adjoint_kernels.hpp"

namespace lr {
LR_INSTANTIATE_BATCH_ADJ(18)
LR_INSTANTIATE_BATCH_ADJ(20)
LR_INSTANTIATE_BATCH_ADJ(22)
LR_INSTANTIATE_BATCH_ADJ(24)
}  // namespace lr
