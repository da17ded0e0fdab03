// Stand-ins for the device-side launch helpers, so that the host ABI layer
// (wkern.cpp) links into a CPU-only sanitizer build.  None of them is reached
// there: every check the driver runs stops before a device is touched.
#include <cstdio>
#include <cstdlib>

#include "wkern_internal.h"

namespace wkern {

[[noreturn]] static void unreachable(const char* name) {
  std::fprintf(stderr, "host ABI check reached %s\n", name);
  std::abort();
}

ContractShape contract_shape(int) { unreachable("contract_shape"); }
hipError_t launch_grad(const DevPlan&, const GradScratch&, const float*, const double*,
                       const void*, float*, double*, hipStream_t) { unreachable("launch_grad"); }
hipError_t launch_hankel_matrix(const DevPlan&, hipStream_t) { unreachable("launch_hankel_matrix"); }
hipError_t prepare_kernels(const DevPlan&) { unreachable("prepare_kernels"); }
hipError_t launch_screen(const DevPlan&, int, int, const float*, const double*, ScreenLayout,
                         hipStream_t) { unreachable("launch_screen"); }
hipError_t launch_contract(const DevPlan&, int, const Tile*, int, hipStream_t) {
  unreachable("launch_contract");
}
hipError_t launch_spline(const DevPlan&, int, int, hipStream_t, double, int32_t*) {
  unreachable("launch_spline");
}
hipError_t launch_resample_truncated(const DevPlan&, const TruncScratch&, double, int32_t*,
                                     int64_t*, void*, hipStream_t) {
  unreachable("launch_resample_truncated");
}
hipError_t launch_resample(const DevPlan&, int, int, void*, hipStream_t) {
  unreachable("launch_resample");
}
hipError_t prepare_resample_kernels(const DevPlan&) { unreachable("prepare_resample_kernels"); }
hipError_t launch_lines_out(const DevPlan&, void*, hipStream_t) { unreachable("launch_lines_out"); }
hipError_t launch_supports(const DevPlan&, const int32_t*, const int32_t*, int32_t*, hipStream_t) {
  unreachable("launch_supports");
}
hipError_t launch_grid(const DevPlan&, int32_t*, const double*, const double*, const double*,
                       const void*, int64_t, const int32_t*, const int64_t*, const int32_t*,
                       const void*, const int64_t*, int, double, void*, hipStream_t) {
  unreachable("launch_grid");
}
hipError_t launch_ps_lines(const DevPlan&, const PsTables&, int, int, const float*,
                           const double*, hipStream_t) {
  unreachable("launch_ps_lines");
}

}  // namespace wkern
