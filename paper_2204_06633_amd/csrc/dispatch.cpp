// Runtime dispatch from the interpolation order to the compiled tap counts.
#include "batch_types.hpp"
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

// (waveform mode, group, workgroup lanes) -> fused kernel instance; tile =
// 2 x lanes link samples per work item.
#define LR_FUSED_CASES(NT, GEN, CALL, FAIL)                                       \
  switch ((wave ? 100000 : 0) + group * 10000 + tile / 2) {                      \
    case 10128: return CALL(NT, GEN, 1, 128, false);                              \
    case 10256: return CALL(NT, GEN, 1, 256, false);                              \
    case 10512: return CALL(NT, GEN, 1, 512, false);                              \
    case 20128: return CALL(NT, GEN, 2, 128, false);                              \
    case 20256: return CALL(NT, GEN, 2, 256, false);                              \
    case 20512: return CALL(NT, GEN, 2, 512, false);                              \
    case 40128: return CALL(NT, GEN, 4, 128, false);                              \
    case 40256: return CALL(NT, GEN, 4, 256, false);                              \
    case 110256: return CALL(NT, GEN, 1, 256, true);                              \
    case 120256: return CALL(NT, GEN, 2, 256, true);                              \
    case 120512: return CALL(NT, GEN, 2, 512, true);                              \
    default: return FAIL;                                                         \
  }

#define LR_LAUNCH_FUSED(NT, GEN, M, B, W) launch_fused_forward<NT, GEN, M, B, W>(a, blocks, s)
#define LR_OCC_FUSED(NT, GEN, M, B, W) fused_occupancy<NT, GEN, M, B, W>()

hipError_t run_fused_forward(int order, int gen, int group, int tile, bool wave,
                             const BatchFwdArgs& a, int blocks, hipStream_t s) {
  // the kernel's rows hold at most fused_halo_cap(group, workgroup) carried
  // samples, and a segment of one tile carries none
  if (a.seg_tiles < 1 || a.HP < 0 || a.HP > fused_halo_cap(group, tile / 2) ||
      (a.seg_tiles > 1) != (a.HP > 0) || (a.HP > 0 && a.HP != tile - a.T_out))
    return hipErrorInvalidValue;
  switch (order) {
#define X(ORD, NT)                                                                        \
  case ORD:                                                                               \
    if (gen == 1) {                                                                       \
      LR_FUSED_CASES(NT, 1, LR_LAUNCH_FUSED, hipErrorInvalidValue)                        \
    } else {                                                                              \
      LR_FUSED_CASES(NT, 2, LR_LAUNCH_FUSED, hipErrorInvalidValue)                        \
    }
    LR_ORDER_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

int fused_blocks_per_cu(int order, int gen, int group, int tile, bool wave) {
  switch (order) {
#define X(ORD, NT)                                                                        \
  case ORD:                                                                               \
    if (gen == 1) {                                                                       \
      LR_FUSED_CASES(NT, 1, LR_OCC_FUSED, 1)                                              \
    } else {                                                                              \
      LR_FUSED_CASES(NT, 2, LR_OCC_FUSED, 1)                                              \
    }
    LR_ORDER_CASES(X)
#undef X
    default: return 1;
  }
}

hipError_t run_batch_tdi_adjoint(int order, int gen, const BatchAdjArgs& a, int64_t n_items,
                                 hipStream_t s) {
  switch (order) {
#define X(ORD, NT) \
  case ORD:        \
    return gen == 1 ? launch_batch_tdi_adjoint<NT, 1>(a, n_items, s) \
                    : launch_batch_tdi_adjoint<NT, 2>(a, n_items, s);
    LR_ORDER_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

hipError_t run_batch_project_adjoint(int order, const BatchAdjArgs& a, int64_t n_items,
                                     int64_t n_sky_items, hipStream_t s) {
  switch (order) {
#define X(ORD, NT) case ORD: return launch_batch_project_adjoint<NT>(a, n_items, n_sky_items, s);
    LR_ORDER_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lr
