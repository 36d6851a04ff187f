// Launch geometry shared by the kernels and the host glue.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "hc_internal.h"

namespace hc {

constexpr int kHistThreads = 512;      // histogram work-group size (8 waves)
constexpr uint64_t kHistMinChunk = 128 * 1024;
constexpr int kHistTargetGroups = 512; // two 64 KiB-LDS groups per CU on 256 CUs

constexpr int kTileThreads = 256;      // encode work-group size (4 waves)
constexpr int kSymPerThread = 16;      // one 16-byte load per thread
constexpr uint32_t kTileSyms = kTileThreads * kSymPerThread;  // 4096 symbols per tile

constexpr int kDecThreads = 256;

struct TileGeom {
    uint64_t n;    // symbols
    uint64_t nb;   // blocks
    uint32_t B;    // symbols per block
    uint32_t tpb;  // tiles per block: ceil(B / kTileSyms)
};

inline TileGeom make_geom(uint64_t n, uint32_t B)
{
    TileGeom g;
    g.n = n;
    g.B = B;
    g.nb = (n + B - 1) / B;
    g.tpb = (B + kTileSyms - 1) / kTileSyms;
    return g;
}

struct EncodeWs {
    uint64_t *counter;  // tile counter (low 32 bits used)
    uint64_t *tstate;   // look-back state per tile
    uint64_t *bstate;   // look-back state per block
};

// Bytes of encode workspace and its carving into arrays.
uint64_t encode_ws_bytes(const TileGeom &g);
EncodeWs carve_encode_ws(void *ws, const TileGeom &g);

hipError_t launch_histogram(const uint8_t *in, uint64_t n, uint64_t *hist, hipStream_t s);
hipError_t launch_encode(const uint8_t *in, const TileGeom &g, const DevTables *tb, uint32_t max_len,
                         uint8_t *out, uint64_t *block_off, uint32_t *sub_idx, uint32_t S,
                         const EncodeWs &ws, uint32_t *err, hipStream_t s);
hipError_t launch_walk(const uint8_t *in, uint64_t in_bytes, uint64_t nb, uint64_t *block_off,
                       uint32_t *err, hipStream_t s);
hipError_t launch_decode(const uint8_t *in, uint64_t in_bytes, uint64_t n, uint32_t B, const DevTables *tb,
                         uint32_t max_len, const uint64_t *block_off, const uint32_t *sub_idx, uint32_t S,
                         uint8_t *out, uint32_t *err, hipStream_t s);

}  // namespace hc
