// Stand-ins for the kernel launchers of drot_kernels.hip in the sanitizer
// build of the host code (tests/test_host_sanitizers.py): the checks there
// never reach a launch, and a launch that happened would fail loudly.
#include <hip/hip_runtime.h>

#include "drot_internal.h"

namespace drot {

hipError_t launch_sweep(int, int, const TileCfg&, const SweepArgs&, hipStream_t, hipEvent_t,
                        hipEvent_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_aux(int, int, const SweepArgs&, hipStream_t, bool, bool) {
  return hipErrorInvalidValue;
}
hipError_t launch_finish(int, const SweepArgs&, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_prep(const SweepArgs&, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_small(int, const SweepArgs&, int64_t, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_maxc(const SweepArgs&, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_batch_step(int, int, const TileCfg&, const SweepArgs*, const uint2*, int64_t,
                             const uint2*, int64_t, int, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_prep_batch(const SweepArgs*, int, hipStream_t) { return hipErrorInvalidValue; }

}  // namespace drot
