// Stand-ins for the kernel launchers of hc_kernels.hip in the host-only
// sanitizer build of the library's C++ (no device code is compiled there):
// every launch reports a runtime error, so a call that gets past its
// argument checks returns HC_ERR_HIP.
#include <hip/hip_runtime_api.h>

#include "hc_kernels.h"

namespace hc {

hipError_t launch_put_jobs(const Job *, uint32_t, uint64_t, Job *, uint64_t *, hipStream_t)
{
    return hipErrorInvalidValue;
}
hipError_t launch_histogram(const JobList &, uint64_t, uint64_t, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_encode(const JobList &, uint64_t, uint32_t, uint32_t, uint32_t, uint32_t, void *, uint32_t *,
                         hipStream_t, uint32_t, bool)
{
    return hipErrorInvalidValue;
}
hipError_t launch_encode_empty(uint64_t *, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_walk(const uint8_t *, uint64_t, uint64_t, uint64_t *, uint32_t *, hipStream_t)
{
    return hipErrorInvalidValue;
}
hipError_t launch_decode_sync(const JobList &, uint64_t, uint32_t, uint32_t, uint32_t *, hipStream_t)
{
    return hipErrorInvalidValue;
}
hipError_t launch_decode(const JobList &, uint64_t, uint32_t, uint32_t, uint32_t, bool, uint32_t *, hipStream_t, bool)
{
    return hipErrorInvalidValue;
}

}  // namespace hc
