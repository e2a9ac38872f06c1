// Stand-ins for the kernel launchers, so that the library's host half
// (argument checks, orbit spline fit, padding rules, batch plans) can be
// built and run on a machine without a GPU under the host sanitizers.  Each
// records that it was reached and launches nothing.
#include "../../paper_2204_06633_amd/csrc/batch_types.hpp"
#include "../../paper_2204_06633_amd/csrc/gb_types.hpp"
#include "../../paper_2204_06633_amd/csrc/internal.hpp"

int g_launches = 0;

namespace lr {
hipError_t run_fill_zero(double*, int64_t, hipStream_t) { ++g_launches; return hipSuccess; }
hipError_t run_sky_finalize(const double*, int64_t, double*, hipStream_t) { ++g_launches; return hipSuccess; }
size_t loglike_workspace_bytes() { return 1024 * sizeof(double); }
hipError_t run_loglike(const double*, const double*, int64_t, double, double*, double*, double*,
                       hipStream_t) { ++g_launches; return hipSuccess; }
hipError_t run_tdi_adjoint(int, int, const TdiAdjArgs&, hipStream_t) { ++g_launches; return hipSuccess; }
hipError_t run_batch_loglike(const double*, const double*, const int64_t*, int64_t, double,
                             double*, double*, const int64_t*, int64_t, double*, hipStream_t) {
  ++g_launches; return hipSuccess;
}
hipError_t run_batch_sky_finalize(const double*, const int64_t*, int64_t, double*, hipStream_t) {
  ++g_launches; return hipSuccess;
}
hipError_t run_forward_prep(int*, const double*, int, int64_t, double*, hipStream_t) {
  ++g_launches; return hipSuccess;
}
hipError_t run_project_adjoint(int, const ProjAdjArgs&, hipStream_t) { ++g_launches; return hipSuccess; }
hipError_t run_project_links(int, const ProjArgs&, hipStream_t) { ++g_launches; return hipSuccess; }
hipError_t run_tdi(int, int, const TdiArgs&, hipStream_t) { ++g_launches; return hipSuccess; }
hipError_t run_fused_forward(int, int, int, int, bool, const BatchFwdArgs&, int, hipStream_t) {
  ++g_launches; return hipSuccess;
}
int fused_blocks_per_cu(int, int, int, int, bool) { return 3; }
hipError_t run_batch_tdi_adjoint(int, int, const BatchAdjArgs&, int64_t, hipStream_t) {
  ++g_launches; return hipSuccess;
}
hipError_t run_batch_project_adjoint(int, const BatchAdjArgs&, int64_t, int64_t, hipStream_t) {
  ++g_launches; return hipSuccess;
}
hipError_t run_gb_batch_finalize(const double*, const int64_t*, const double*, const int64_t*,
                                 const double*, int64_t, double*, hipStream_t) {
  ++g_launches; return hipSuccess;
}
}  // namespace lr
