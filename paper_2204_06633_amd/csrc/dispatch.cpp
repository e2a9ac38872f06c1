// Runtime dispatch from the interpolation order to the compiled tap counts.
#include "internal.hpp"

namespace lr {

#define LR_ORDER_CASES(X) \
  X(1, 2) X(3, 4) X(5, 6) X(7, 8) X(9, 10) X(11, 12) X(13, 14) X(15, 16) \
  X(17, 18) X(19, 20) X(21, 22) X(23, 24) X(25, 26) X(27, 28) X(29, 30) X(31, 32)

hipError_t run_project_links(int order, const ProjArgs& a, hipStream_t s) {
  switch (order) {
#define X(ORD, NT) case ORD: return launch_project<NT>(a, s);
    LR_ORDER_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

hipError_t run_tdi(int order, int gen, const TdiArgs& a, hipStream_t s) {
  switch (order) {
#define X(ORD, NT) case ORD: return launch_tdi<NT>(a, gen, s);
    LR_ORDER_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

hipError_t run_tdi_adjoint(int order, int gen, const TdiAdjArgs& a, hipStream_t s) {
  switch (order) {
#define X(ORD, NT) case ORD: return launch_tdi_adjoint<NT>(a, gen, s);
    LR_ORDER_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

hipError_t run_project_adjoint(int order, const ProjAdjArgs& a, hipStream_t s) {
  switch (order) {
#define X(ORD, NT) case ORD: return launch_project_adjoint<NT>(a, s);
    LR_ORDER_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lr
