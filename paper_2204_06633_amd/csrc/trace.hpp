// Named ranges for rocprofv3's marker trace (--marker-trace): every C-ABI
// call that does device work opens a roctx range named after the call and
// closes it on return, so a trace shows which call issued which kernels and
// copies.  With no tool attached a push / pop pair is a cheap no-op.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace lr {

class CallRange {
 public:
  explicit CallRange(const char* name) { roctxRangePushA(name); }
  ~CallRange() { roctxRangePop(); }
  CallRange(const CallRange&) = delete;
  CallRange& operator=(const CallRange&) = delete;
};

}  // namespace lr

#define LR_CALL_RANGE() const ::lr::CallRange lr_call_range_(__func__)
