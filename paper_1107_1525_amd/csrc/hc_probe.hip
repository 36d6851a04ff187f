// Roofline probes: a streaming copy and a streaming read of device memory.
// They give the achievable side of the HBM roofline the codec kernels are
// measured against: the rate plain, fully coalesced 16-byte accesses reach on
// this device (each wave instruction covers 1 KiB of contiguous memory),
// marked non-temporal.  The shapes (a 32 KiB tile per copy group; 1024
// reading groups with 16 loads in flight per thread, each over a contiguous
// range) and the cache policy were the fastest of sweeps over loads in
// flight, group counts, strided or contiguous ranges and non-temporal or
// plain accesses on MI355X.  They are measurement helpers, not part of the
// coding path.
#include <hip/hip_runtime.h>

#include "hc.h"

namespace {

typedef uint32_t pv4 __attribute__((ext_vector_type(4)));
constexpr uint32_t kProbeThreads = 256;
constexpr uint32_t kCopyUnroll = 8;            // a copy group moves one 32 KiB tile: 8 loads per thread
constexpr uint32_t kReadUnroll = 16;           // 16 loads in flight per reading thread
constexpr uint32_t kReadMaxGroups = 1024;      // 4 per CU, each streaming a contiguous range
constexpr uint64_t kCopyTile = (uint64_t)kProbeThreads * kCopyUnroll;  // vectors per copy group

// Work-group g copies vectors [g * kCopyTile, +kCopyTile): all loads first,
// then all stores; one tile per group, so thousands of groups stream at once.
__global__ __launch_bounds__(kProbeThreads) void k_probe_copy(const pv4 *__restrict__ src, pv4 *__restrict__ dst,
                                                               uint64_t nvec)
{
    const uint64_t base = (uint64_t)blockIdx.x * kCopyTile + threadIdx.x;
    if (base + (kCopyUnroll - 1) * kProbeThreads < nvec) {
        pv4 v[kCopyUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kCopyUnroll; ++u) v[u] = __builtin_nontemporal_load(&src[base + u * kProbeThreads]);
#pragma unroll
        for (uint32_t u = 0; u < kCopyUnroll; ++u) __builtin_nontemporal_store(v[u], &dst[base + u * kProbeThreads]);
    } else {
        for (uint32_t u = 0; u < kCopyUnroll; ++u)
            if (base + u * kProbeThreads < nvec) dst[base + u * kProbeThreads] = src[base + u * kProbeThreads];
    }
}

// Work-group g reads the contiguous range [g * per_group, +per_group) with
// kReadUnroll loads in flight per thread and folds the words into *sink with
// xor (one atomic per wave; the value only keeps the reads from being
// removed).  Few groups, so the atomics stay negligible.
__global__ __launch_bounds__(kProbeThreads) void k_probe_read(const pv4 *__restrict__ src, uint64_t nvec,
                                                               uint64_t per_group, uint32_t *sink)
{
    const uint64_t beg = (uint64_t)blockIdx.x * per_group;
    const uint64_t end = beg + per_group < nvec ? beg + per_group : nvec;
    uint32_t x = 0;
    uint64_t i = beg + threadIdx.x;
    for (; i + (kReadUnroll - 1) * kProbeThreads < end; i += kReadUnroll * kProbeThreads) {
        pv4 v[kReadUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kReadUnroll; ++u) v[u] = __builtin_nontemporal_load(&src[i + u * kProbeThreads]);
#pragma unroll
        for (uint32_t u = 0; u < kReadUnroll; ++u) x ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    for (; i < end; i += kProbeThreads) {
        const pv4 v = src[i];
        x ^= v.x ^ v.y ^ v.z ^ v.w;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x ^= __shfl_xor(x, o, 64);
    if ((threadIdx.x & 63u) == 0) atomicXor(sink, x);
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

}  // namespace

extern "C" hc_status hc_probe_copy(const void *d_src, void *d_dst, uint64_t n, void *stream)
{
    if (n % 16 != 0) return HC_ERR_INVALID_ARG;
    if (n == 0) return HC_OK;
    if (!d_src || !d_dst || !aligned16(d_src) || !aligned16(d_dst)) return HC_ERR_INVALID_ARG;
    const uintptr_t a = (uintptr_t)d_src, b = (uintptr_t)d_dst;
    if (a < b + n && b < a + n) return HC_ERR_INVALID_ARG;  // overlapping ranges
    const uint64_t nvec = n / 16;
    const uint64_t groups = (nvec + kCopyTile - 1) / kCopyTile;
    if (groups > 0x7fffffffull) return HC_ERR_INVALID_ARG;  // beyond one launch's grid (32 TiB)
    k_probe_copy<<<dim3((uint32_t)groups), kProbeThreads, 0, (hipStream_t)stream>>>((const pv4 *)d_src,
                                                                                    (pv4 *)d_dst, nvec);
    return hipGetLastError() == hipSuccess ? HC_OK : HC_ERR_HIP;
}

extern "C" hc_status hc_probe_read(const void *d_src, uint64_t n, uint32_t *d_sink, void *stream)
{
    if (n % 16 != 0 || !d_sink || ((uintptr_t)d_sink & 3u)) return HC_ERR_INVALID_ARG;
    if (n == 0) return HC_OK;
    if (!d_src || !aligned16(d_src)) return HC_ERR_INVALID_ARG;
    const uint64_t nvec = n / 16;
    const uint64_t per_unroll = (uint64_t)kProbeThreads * kReadUnroll;
    uint64_t groups = (nvec + per_unroll - 1) / per_unroll;
    groups = groups < kReadMaxGroups ? groups : kReadMaxGroups;
    const uint64_t per_group = (nvec + groups - 1) / groups;
    k_probe_read<<<dim3((uint32_t)groups), kProbeThreads, 0, (hipStream_t)stream>>>((const pv4 *)d_src, nvec,
                                                                                    per_group, d_sink);
    return hipGetLastError() == hipSuccess ? HC_OK : HC_ERR_HIP;
}
