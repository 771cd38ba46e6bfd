// The device plan builder's kernel launcher, absent from a host-only build: the host
// builder never calls it.
#include "../../paper_2201_02309_amd/csrc/kernels.hpp"

namespace kats {
hipError_t launch_plan_device(const DevPlanArgs &, const DevPlanPtrs &, hipStream_t) {
    return hipErrorNotSupported;
}
}  // namespace kats
