// C ABI entry points: argument checks, then kernel launches on the caller's
// stream.  See include/hc.h for the contract of every call.
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "hc_internal.h"
#include "hc_kernels.h"

using namespace hc;

namespace {

bool aligned(const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

bool valid_block_size(uint32_t B) { return B >= 16 && B <= (1u << 26) && (B % 16) == 0; }

bool valid_sub_block(uint32_t S) { return S == 0 || (S % 16) == 0; }

hc_status hip_status(hipError_t e) { return e == hipSuccess ? HC_OK : HC_ERR_HIP; }

}  // namespace

extern "C" const char *hc_status_str(int status)
{
    switch (status) {
    case HC_OK: return "HC_OK";
    case HC_ERR_INVALID_ARG: return "HC_ERR_INVALID_ARG";
    case HC_ERR_NO_SPACE: return "HC_ERR_NO_SPACE";
    case HC_ERR_HIP: return "HC_ERR_HIP";
    case HC_ERR_SYMBOL_ABSENT: return "HC_ERR_SYMBOL_ABSENT";
    case HC_ERR_BLOCK_OVERFLOW: return "HC_ERR_BLOCK_OVERFLOW";
    case HC_ERR_CORRUPT: return "HC_ERR_CORRUPT";
    case HC_ERR_CODE_TOO_LONG: return "HC_ERR_CODE_TOO_LONG";
    default: return "HC_ERR_UNKNOWN";
    }
}

extern "C" int hc_version(void) { return 100; }

extern "C" hc_status hc_histogram(const uint8_t *d_in, uint64_t n, uint64_t *d_hist, void *stream)
{
    if (!d_hist || !aligned(d_hist, 8)) return HC_ERR_INVALID_ARG;
    if (n > 0 && (!d_in || !aligned(d_in, 16))) return HC_ERR_INVALID_ARG;
    return hip_status(launch_histogram(d_in, n, d_hist, static_cast<hipStream_t>(stream)));
}

namespace {

// The codebook must be the canonical code of its own lengths.
hc_status validate_codebook(const hc_codebook *cb)
{
    hc_codebook check;
    hc_status st = canonical_from_lengths(cb->len, &check);
    if (st != HC_OK) return st;
    if (check.max_len != cb->max_len || check.nsym != cb->nsym ||
        memcmp(check.code, cb->code, sizeof(check.code)) != 0)
        return HC_ERR_INVALID_ARG;
    return HC_OK;
}

void release(hc_cb_dev_s *h)
{
    if (h->d_tables) (void)hipFree(h->d_tables);
    if (h->staging) (void)hipHostFree(h->staging);
    if (h->copy_done) (void)hipEventDestroy(static_cast<hipEvent_t>(h->copy_done));
    free(h);
}

}  // namespace

extern "C" hc_status hc_codebook_upload(const hc_codebook *cb, hc_cb_handle *out)
{
    if (!cb || !out) return HC_ERR_INVALID_ARG;
    *out = nullptr;
    hc_status st = validate_codebook(cb);
    if (st != HC_OK) return st;
    hc_cb_dev_s *h = static_cast<hc_cb_dev_s *>(calloc(1, sizeof(hc_cb_dev_s)));
    if (!h) return HC_ERR_INVALID_ARG;
    h->host = *cb;
    hipEvent_t ev = nullptr;
    if (hipGetDevice(&h->device) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&h->staging), sizeof(DevTables), hipHostMallocDefault) !=
            hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&h->d_tables), sizeof(DevTables)) != hipSuccess ||
        hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        release(h);
        return HC_ERR_HIP;
    }
    h->copy_done = ev;
    build_dev_tables(*cb, h->staging);
    if (hipMemcpy(h->d_tables, h->staging, sizeof(DevTables), hipMemcpyHostToDevice) != hipSuccess) {
        release(h);
        return HC_ERR_HIP;
    }
    *out = h;
    return HC_OK;
}

extern "C" hc_status hc_codebook_update(hc_cb_handle h, const hc_codebook *cb, void *stream)
{
    if (!h || !cb) return HC_ERR_INVALID_ARG;
    hc_status st = validate_codebook(cb);
    if (st != HC_OK) return st;
    hipEvent_t ev = static_cast<hipEvent_t>(h->copy_done);
    if (hipEventSynchronize(ev) != hipSuccess) return HC_ERR_HIP;  // staging no longer being read
    build_dev_tables(*cb, h->staging);
    h->host = *cb;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(h->d_tables, h->staging, sizeof(DevTables), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipEventRecord(ev, s) != hipSuccess)
        return HC_ERR_HIP;
    return HC_OK;
}

extern "C" hc_status hc_codebook_destroy(hc_cb_handle cb)
{
    if (!cb) return HC_OK;
    hipError_t e = hipDeviceSynchronize();
    release(cb);
    return hip_status(e);
}

extern "C" uint64_t hc_encode_bound(uint64_t n, uint32_t block_size, uint32_t max_len)
{
    if (block_size == 0 || max_len > (uint32_t)kMaxLen) return 0;
    const uint64_t full = n / block_size, rest = n % block_size;
    const uint64_t per_full = 4 + 4 * (((uint64_t)block_size * max_len + 31) / 32);
    uint64_t total = full * per_full;
    if (rest) total += 4 + 4 * ((rest * max_len + 31) / 32);
    return total;
}

extern "C" uint64_t hc_encode_workspace_bytes(uint64_t n, uint32_t block_size)
{
    if (block_size == 0) return 0;
    return encode_ws_bytes(make_geom(n, block_size));
}

extern "C" uint64_t hc_sub_index_entries(uint64_t n, uint32_t block_size, uint32_t sub_block)
{
    if (block_size == 0 || sub_block == 0) return 0;
    const uint64_t nb = (n + block_size - 1) / block_size;
    return nb * ((block_size + sub_block - 1) / sub_block);
}

extern "C" hc_status hc_encode_blocks(const uint8_t *d_in, uint64_t n, uint32_t block_size, hc_cb_handle cb,
                                      uint8_t *d_out, uint64_t out_cap, uint64_t *d_block_off,
                                      uint32_t *d_sub_idx, uint32_t sub_block, void *d_ws,
                                      uint64_t ws_bytes, uint32_t *d_err, void *stream)
{
    if (!valid_block_size(block_size) || !valid_sub_block(sub_block) || !cb || !d_block_off ||
        !aligned(d_block_off, 8))
        return HC_ERR_INVALID_ARG;
    if ((d_sub_idx == nullptr) != (sub_block == 0)) return HC_ERR_INVALID_ARG;
    if (d_sub_idx && !aligned(d_sub_idx, 4)) return HC_ERR_INVALID_ARG;
    const TileGeom g = make_geom(n, block_size);
    if (n > 0) {
        if (!d_in || !aligned(d_in, 16) || !d_out || !aligned(d_out, 16) || !d_ws || !aligned(d_ws, 8))
            return HC_ERR_INVALID_ARG;
        if (cb->host.max_len == 0) return HC_ERR_INVALID_ARG;  // no code for any symbol
        if (out_cap < hc_encode_bound(n, block_size, cb->host.max_len)) return HC_ERR_NO_SPACE;
        if (ws_bytes < encode_ws_bytes(g)) return HC_ERR_NO_SPACE;
        if (g.nb * g.tpb > 0x7FFFFFFFull) return HC_ERR_INVALID_ARG;  // grid limit
    }
    const EncodeWs ws = n > 0 ? carve_encode_ws(d_ws, g) : EncodeWs{nullptr, nullptr, nullptr};
    return hip_status(launch_encode(d_in, g, cb->d_tables, cb->host.max_len, d_out, d_block_off, d_sub_idx,
                                    sub_block, ws, d_err, static_cast<hipStream_t>(stream)));
}

extern "C" hc_status hc_walk_blocks(const uint8_t *d_in, uint64_t in_bytes, uint64_t nb, uint64_t *d_block_off,
                                    uint32_t *d_err, void *stream)
{
    if (!d_block_off || !aligned(d_block_off, 8)) return HC_ERR_INVALID_ARG;
    if (in_bytes > 0 && (!d_in || !aligned(d_in, 4) || (in_bytes & 3))) return HC_ERR_INVALID_ARG;
    return hip_status(launch_walk(d_in, in_bytes, nb, d_block_off, d_err, static_cast<hipStream_t>(stream)));
}

extern "C" hc_status hc_decode_blocks(const uint8_t *d_in, uint64_t in_bytes, uint64_t n, uint32_t block_size,
                                      hc_cb_handle cb, const uint64_t *d_block_off, const uint32_t *d_sub_idx,
                                      uint32_t sub_block, uint8_t *d_out, uint32_t *d_err, void *stream)
{
    if (!valid_block_size(block_size) || !valid_sub_block(sub_block) || !cb) return HC_ERR_INVALID_ARG;
    if ((d_sub_idx == nullptr) != (sub_block == 0)) return HC_ERR_INVALID_ARG;
    if (n == 0) return HC_OK;
    if (!d_in || !aligned(d_in, 16) || !d_block_off || !aligned(d_block_off, 8) || !d_out ||
        !aligned(d_out, 16) || (d_sub_idx && !aligned(d_sub_idx, 4)))
        return HC_ERR_INVALID_ARG;
    if (cb->host.max_len == 0) return HC_ERR_INVALID_ARG;
    const uint64_t nb = (n + block_size - 1) / block_size;
    const uint64_t lanes = nb * (d_sub_idx ? (block_size + sub_block - 1) / sub_block : 1);
    if ((lanes + kDecThreads - 1) / kDecThreads > 0x7FFFFFFFull) return HC_ERR_INVALID_ARG;
    if (in_bytes & 3) return HC_ERR_INVALID_ARG;
    return hip_status(launch_decode(d_in, in_bytes, n, block_size, cb->d_tables, cb->host.max_len, d_block_off,
                                    d_sub_idx, sub_block, d_out, d_err, static_cast<hipStream_t>(stream)));
}
