// Batched adjoint kernels for tap counts 26, 28, 30, 32.
#include "batch_adjoint_kernels.hpp"

namespace lr {
LR_INSTANTIATE_BATCH_ADJ(26)
LR_INSTANTIATE_BATCH_ADJ(28)
LR_INSTANTIATE_BATCH_ADJ(30)
LR_INSTANTIATE_BATCH_ADJ(32)
}  // namespace lr
