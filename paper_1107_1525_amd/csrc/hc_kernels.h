// Launch geometry and job descriptors shared by the kernels and the host glue.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "hc_internal.h"

namespace hc {

constexpr int kHistThreads = 512;      // histogram work-group size (8 waves)
constexpr uint64_t kHistMinChunk = 128 * 1024;
constexpr int kHistTargetGroups = 512; // two 64 KiB-LDS groups per CU on 256 CUs

constexpr int kTileThreads = 256;      // encode work-group size (4 waves)
constexpr uint32_t kQuadSyms = 16;     // symbols of one 16-byte load
constexpr uint32_t kTileSyms = kTileThreads * kQuadSyms;  // tile of one load per thread

constexpr int kDecThreads = 256;

// One buffer of a launch.  A launch covers one or more jobs; its launch units
// (histogram chunks, encode tiles, decode work-groups) are numbered job after
// job, and unit_begin is the first unit of this job.
struct Job {
    const uint8_t *in;     // histogram/encode: the symbols; decode: the stream
    uint64_t n;            // symbols
    uint64_t in_bytes;     // decode: stream bytes
    const DevTables *tb;   // encode/decode: the job's code tables
    uint8_t *out;          // encode: the stream; decode: the symbols
    uint64_t *block_off;   // encode: written; decode: read
    uint32_t *sub_idx;     // sub-block index or null
    uint64_t *hist;        // histogram: 256 counts
    uint64_t unit_begin;   // first launch unit of the job
};

// The jobs of a launch: a device array, or a single job passed by value.
struct JobList {
    const Job *jobs;         // device array of 'count' jobs, or null when count == 1
    const uint64_t *starts;  // device array: unit_begin of every job, then the total
    uint32_t count;
    Job one;
};

inline uint64_t num_blocks(uint64_t n, uint32_t B) { return (n + B - 1) / B; }
// Symbols of a decode lane's chunk: the sub-block stride S with an index;
// without one, kCopyChunkSyms for a complete 8-bit code (every code has 8
// bits, so chunk c of a block starts at payload bit 8 * S_eff * c and needs
// no index), else the whole block.
constexpr uint32_t kCopyChunkSyms = 128;
inline uint32_t decode_chunk(uint32_t B, uint32_t S, bool with_index, bool complete8)
{
    if (with_index) return S;
    if (complete8) return B < kCopyChunkSyms ? B : kCopyChunkSyms;
    return B;
}
// Loads (16 symbols each) per encode thread: a tile is qpt * 4096 symbols.
// Large tiles give each work-group more bytes to pack per fixed set-up cost
// (tables, the tile's position, the next tile's first symbols); they need
// qpt * 4096 * max_len bits of LDS, so long codes keep the small tile.
inline uint32_t encode_qpt(uint32_t B, uint32_t max_len)
{
    if (max_len > (uint32_t)kPackedMaxLen) return 1;
    if (B >= 4 * kTileSyms && max_len <= 16) return 4;
    if (B >= 2 * kTileSyms) return 2;
    return 1;
}
inline uint32_t tiles_per_block(uint32_t B, uint32_t qpt)
{
    const uint32_t t = qpt * kTileSyms;
    return (B + t - 1) / t;
}
inline uint64_t hist_chunk(uint64_t total)
{
    uint64_t chunk = (total + kHistTargetGroups - 1) / kHistTargetGroups;
    chunk = (chunk + 15) & ~uint64_t(15);
    if (chunk < kHistMinChunk) chunk = kHistMinChunk;
    if (chunk > (1ull << 30)) chunk = 1ull << 30;  // keeps every LDS counter below 2^32
    return chunk;
}

// Encode scratch, in bytes, for 'tiles' tiles of qpt * 4096 symbols: the bit
// count and the in-block bit position of every tile (u32 each), then, when
// qpt >= 2, the bit count of every thread of every tile (u16), which the
// length pass hands to the packing pass.
inline uint64_t encode_scratch_bytes(uint64_t tiles, uint32_t qpt)
{
    return tiles * (8ull + (qpt >= 2 ? 2ull * kTileThreads : 0ull));
}
// The most any code needs for nb blocks of B symbols (every tile shape B allows).
inline uint64_t encode_scratch_bound(uint64_t nb, uint32_t B)
{
    uint64_t most = 0;
    for (uint32_t qpt = 1; qpt <= encode_qpt(B, 1); qpt *= 2) {
        const uint64_t b = encode_scratch_bytes(nb * tiles_per_block(B, qpt), qpt);
        most = b > most ? b : most;
    }
    return most;
}

// Writes a job table and its start units (then 'total') to device memory
// with kernel launches that carry the jobs as arguments: nothing waits for
// the stream and the host array may be reused when the call returns.
hipError_t launch_put_jobs(const Job *jobs, uint32_t count, uint64_t total, Job *d_jobs, uint64_t *d_starts,
                           hipStream_t s);
hipError_t launch_histogram(const JobList &jl, uint64_t units, uint64_t chunk, hipStream_t s);
// Encode steps (bit mask): the length pass, the offset scan, the packing.
constexpr uint32_t kStepLengths = 1, kStepOffsets = 2, kStepPack = 4, kStepAll = 7;
// complete8: every job has a complete 8-bit code (the length pass is left
// out: each symbol costs 8 bits).
hipError_t launch_encode(const JobList &jl, uint64_t tiles, uint32_t B, uint32_t qpt, uint32_t max_len, uint32_t S,
                         void *scratch, uint32_t *err, hipStream_t s, uint32_t steps, bool complete8);
hipError_t launch_encode_empty(uint64_t *block_off, hipStream_t s);
hipError_t launch_walk(const uint8_t *in, uint64_t in_bytes, uint64_t nb, uint64_t *block_off,
                       uint32_t *err, hipStream_t s);
// Decode without the sub-block index: one work-group per block of every job
// (grid = blocks, the jobs' total; max_len: their longest code).
hipError_t launch_decode_sync(const JobList &jl, uint64_t blocks, uint32_t B, uint32_t max_len, uint32_t *err,
                              hipStream_t s);
// complete8: every job has a complete 8-bit code (all 256 bytes coded with 8
// bits), decoded by the copy form alone.
hipError_t launch_decode(const JobList &jl, uint64_t groups, uint32_t B, uint32_t max_len, uint32_t S,
                         bool with_index, uint32_t *err, hipStream_t s, bool complete8 = false);

}  // namespace hc
