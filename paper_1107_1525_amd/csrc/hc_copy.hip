// A streaming copy between device memory and pinned host memory that does
// not go through the runtime's copy engines: one work-group per CU, each
// streaming a contiguous range with 16 dwordx4 loads in flight per thread
// and writing straight into the destination (pinned host memory is reached
// over PCIe).  The small grid leaves the CUs to coding kernels running beside
// it.  Both ranges must be device-accessible at their own addresses (device
// memory, or host memory pinned by the HIP runtime), each inside one
// allocation; the call asks the runtime before launching and refuses
// anything else, pageable host memory included.
#include <hip/hip_runtime.h>

#include "hc.h"

namespace {

typedef uint32_t cv4 __attribute__((ext_vector_type(4)));
constexpr uint32_t kCopyThreads = 256;
constexpr uint32_t kCopyUnroll = 16;
constexpr uint32_t kCopyGroups = 256;  // one per CU

__global__ __launch_bounds__(kCopyThreads) void k_copy(const cv4 *__restrict__ src, cv4 *__restrict__ dst,
                                                        uint64_t nvec, uint64_t per_group)
{
    const uint64_t beg = (uint64_t)blockIdx.x * per_group;
    const uint64_t end = beg + per_group < nvec ? beg + per_group : nvec;
    uint64_t i = beg + threadIdx.x;
    for (; i + (kCopyUnroll - 1) * kCopyThreads < end; i += kCopyUnroll * kCopyThreads) {
        cv4 v[kCopyUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kCopyUnroll; ++u) v[u] = src[i + u * kCopyThreads];
#pragma unroll
        for (uint32_t u = 0; u < kCopyUnroll; ++u) dst[i + u * kCopyThreads] = v[u];
    }
    for (; i < end; i += kCopyThreads) dst[i] = src[i];
}

// The runtime knows [p, p + n) as part of one allocation (device memory or
// its own pinned host memory), and the device reaches it at the same
// address.  Asking about the two ends alone would accept a range whose ends
// lie in two allocations with unmapped memory between them.
bool device_visible(const void *p, uint64_t n)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();  // an unknown (pageable) pointer: clear the error it leaves
        return false;
    }
    if (a.type != hipMemoryTypeHost && a.type != hipMemoryTypeDevice) return false;
    if (a.devicePointer != p) return false;
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, const_cast<void *>(p)) != hipSuccess || !base) {
        (void)hipGetLastError();
        return false;
    }
    const uintptr_t b = (uintptr_t)base, q = (uintptr_t)p;
    return q >= b && q - b <= size && n <= size - (q - b);
}

}  // namespace

extern "C" hc_status hc_copy(const void *d_src, void *d_dst, uint64_t n, void *stream)
{
    if (n % 16 != 0) return HC_ERR_INVALID_ARG;
    if (n == 0) return HC_OK;
    if (!d_src || !d_dst || ((uintptr_t)d_src & 15u) || ((uintptr_t)d_dst & 15u)) return HC_ERR_INVALID_ARG;
    const uintptr_t a = (uintptr_t)d_src, b = (uintptr_t)d_dst;
    if (a < b + n && b < a + n) return HC_ERR_INVALID_ARG;  // overlapping ranges
    const uint8_t *s8 = static_cast<const uint8_t *>(d_src);
    uint8_t *d8 = static_cast<uint8_t *>(d_dst);
    if (!device_visible(s8, n) || !device_visible(d8, n)) return HC_ERR_INVALID_ARG;
    const uint64_t nvec = n / 16;
    const uint64_t per_unroll = (uint64_t)kCopyThreads * kCopyUnroll;
    uint64_t groups = (nvec + per_unroll - 1) / per_unroll;
    groups = groups < kCopyGroups ? groups : kCopyGroups;
    const uint64_t per_group = (nvec + groups - 1) / groups;
    k_copy<<<dim3((uint32_t)groups), kCopyThreads, 0, (hipStream_t)stream>>>((const cv4 *)d_src, (cv4 *)d_dst, nvec,
                                                                            per_group);
    return hipGetLastError() == hipSuccess ? HC_OK : HC_ERR_HIP;
}
