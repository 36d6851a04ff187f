// hc_encode_blocks_noalloc: block encoding whose scratch is a file-scope
// device array instead of a caller workspace, for callers that may not
// allocate (code under stream capture, tight serving loops).
//
// The encoder's scratch (per tile its bit count and in-block bit position,
// per thread of a large tile its bit count) lives in 'scratch' below.  Each
// GPU the library runs on holds its own copy of the array at its own address
// until the process ends; host code learns that address once per device with
// hipGetSymbolAddress and passes it to the kernels, never the array's name
// (which in host code is only a stand-in for the device symbol).
#include <hip/hip_runtime.h>

#include <mutex>

#include "hc_internal.h"

namespace {

constexpr uint64_t kScratchBytes = HC_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "whole 256-byte granules");

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];  // device address of 'scratch' on each device, once looked up

// The address of this device's copy of 'scratch' (nullptr if the runtime
// cannot give it).  The lookup runs once per device, with that device current.
void *scratch_on(int dev)
{
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_ptr[dev] = p;
    }
    return g_ptr[dev];
}

}  // namespace

extern "C" hc_status hc_encode_blocks_noalloc(const uint8_t *d_in, uint64_t n, uint32_t block_size, hc_cb_handle cb,
                                              uint8_t *d_out, uint64_t out_cap, uint64_t *d_block_off,
                                              uint32_t *d_sub_idx, uint32_t sub_block, uint32_t *d_err, void *stream)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return HC_ERR_HIP;
    if (dev >= kMaxDevices) return HC_ERR_INVALID_ARG;
    void *ws = scratch_on(dev);
    if (!ws) return HC_ERR_HIP;
    // the same checks and launches as hc_encode_blocks: a call whose scratch
    // need exceeds the array returns HC_ERR_NO_SPACE and launches nothing
    return hc::encode_blocks_ws(d_in, n, block_size, cb, d_out, out_cap, d_block_off, d_sub_idx, sub_block, ws,
                                kScratchBytes, d_err, stream);
}
