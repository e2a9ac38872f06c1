// The build-time tuning switches this library was compiled with, as one
// "NAME=value;..." string (lr_build_config).  The kernel headers define the
// product defaults; a variant build (-D on every unit) reports its own
// values, so a caller or a test can tell the two apart from the binary.
#include "adjoint_kernels.hpp"
#include "batch_kernels.hpp"
#include "fd_types.hpp"
#include "forward_kernels.hpp"

#define LR_STR2(x) #x
#define LR_STR(x) LR_STR2(x)
#define LR_ITEM(name) #name "=" LR_STR(name) ";"

extern "C" const char* lr_build_config(void) {
  return LR_ITEM(LR_PROJ_PIPE) LR_ITEM(LR_PROJ_MIN_WAVES) LR_ITEM(LR_TDI_MIN_WAVES)
      LR_ITEM(LR_FUSED_MIN_WAVES) LR_ITEM(LR_FUSED2_MIN_WAVES) LR_ITEM(LR_FUSED2W_MIN_WAVES)
          LR_ITEM(LR_TDI_CARRY_MIN_WAVES) LR_ITEM(LR_PADJ_CARRY_MIN_WAVES) LR_ITEM(LR_TDI_CARRY_KEEP_NU)
              LR_ITEM(LR_TDI_ADJ_FOLD) LR_ITEM(LR_PADJ_MIN_WAVES) LR_ITEM(LR_SKY_MIN_WAVES)
                  LR_ITEM(LR_FD_LS_EXTRA);
}
