// Host-only stand-ins for the kernel launchers of kernels.hip, so that the
// planner sources link into a CPU program built with the address, undefined
// behaviour or thread sanitizer.  Plan dry runs never launch anything; a call
// here would be a bug, so each one aborts.
#include <cstdlib>
#include "../../paper_2107_02671_amd/csrc/internal.h"
namespace nnfft {
hipError_t launch_nfft(const PlanDev &, bool, const void *, void *, hipStream_t) { std::abort(); }
hipError_t launch_exec(const PlanDev &, const void *, void *, hipStream_t, hipEvent_t *) { std::abort(); }
hipError_t launch_scale_by_weights(int, const double *, const void *, void *, int64_t, hipStream_t) { std::abort(); }
hipError_t launch_exec_batch(int, const PlanDev *const *, const PlanDev *const *, const void *const *,
                             void *const *, hipStream_t)
{
    std::abort();
}
}  // namespace nnfft
