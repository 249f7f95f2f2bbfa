// Host-only stand-ins for the kernel launchers of kernels.hip and
// plan_device.hip, so that the planner sources link into a CPU program built
// with the address, undefined behaviour or thread sanitizer.  Plan dry runs
// never launch anything; a call here would be a bug, so each one aborts.
#include <cstdlib>
#include "../../paper_2107_02671_amd/csrc/internal.h"
namespace nnfft {
hipError_t launch_nfft(const PlanDev &, bool, const void *, void *, hipStream_t) { std::abort(); }
hipError_t launch_exec(const PlanDev &, const void *, void *, hipStream_t, KernelTimes *) { std::abort(); }
hipError_t launch_scale_by_weights(int, const double *, const void *, void *, int64_t, hipStream_t) { std::abort(); }
hipError_t launch_sinc_middle(const PlanDev &, const SincMidArgs &, const PlanDev &, const void *, void *, hipStream_t)
{
    std::abort();
}
hipError_t launch_exec_batch(int, const PlanDev *const *, const PlanDev *const *, const void *const *,
                             void *const *, hipStream_t)
{
    std::abort();
}
hipError_t launch_exec_static(const PlanDev &, const ExecScratch &, const void *, void *, hipStream_t)
{
    std::abort();
}
size_t static_scratch_need(const ExecScratch &) { std::abort(); }
const char *kernel_name(int) { std::abort(); }
int kernel_stage(int) { std::abort(); }
bool device_sort_fits(int64_t, int64_t, int64_t) { std::abort(); }
size_t device_sort_tmp_bytes(int64_t) { std::abort(); }
hipError_t device_sort_nodes(const double *, int64_t, double, int64_t, int64_t, int64_t, int32_t *, int32_t *, void *,
                             int32_t **, hipStream_t)
{
    std::abort();
}
hipError_t device_sorted_records(const double *, const int32_t *, int64_t, double, bool, int32_t *, double *, PtRec *,
                                 hipStream_t)
{
    std::abort();
}
hipError_t device_gather(const double *, const int64_t *, int64_t, double *, hipStream_t) { std::abort(); }
hipError_t device_transposed_records(const double *, const int32_t *, double, const Item *, int64_t, int, PtRec *,
                                     hipStream_t)
{
    std::abort();
}
bool device_sort_pair_fits(const SortSide &, const SortSide &) { std::abort(); }
hipError_t device_records_pair(bool, const RecSide &, const RecSide &, hipStream_t) { std::abort(); }
hipError_t device_gather_pair(const double *, const int64_t *, int64_t, double *, const double *, const int64_t *,
                              int64_t, double *, hipStream_t)
{
    std::abort();
}
hipError_t device_sort_node_pair(const SortSide &, const SortSide &, void *, int32_t **, int32_t **, hipStream_t)
{
    std::abort();
}
}  // namespace nnfft
