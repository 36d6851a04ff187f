// HIP kernels for gfx950 (CDNA4, wave64) of the block-decomposed Huffman codec.
//
//   k_hist         symbol counts (paper section 2) with LDS-privatised
//                  sub-histograms, one replica per lane of a wavefront
//   k_count        length pass (section 2.1): bits of every tile of 4096 * QPT
//                  symbols (a tile never crosses a block boundary)
//   k_offsets      offset pass (section 2.1: the table of where each block
//                  begins): each tile's bit position inside its block and
//                  each block's byte offset in the stream, one work-group per
//                  stream
//   k_encode       bit packing (section 2.1, Fig. 3-4): a tile's code words
//                  OR-ed into LDS words, stored coalesced at the block's offset
//                  in the stream with the header and zero pad
//   k_walk         offset table rebuilt from the length delimiters
//   k_decode_stage table decode (sections 2.1 and 3.2) with the sub-block
//                  index, S <= 128, codes <= 24 bits: a wave stages its 64
//                  chunks' words in LDS with coalesced loads, one lane decodes
//                  each chunk, output stored through LDS
//   k_decode_ring  the same decode for larger S or none, one lane per chunk
//                  of S symbols (or per block), whole 128-byte lines in from
//                  HBM through an LDS ring per lane; and the copy form of
//                  complete 8-bit codes
//   k_decode_sync  decode without the index: a block's pieces decoded in
//                  parallel from their first bits, then again from where the
//                  left neighbour's codes end until every piece starts on a
//                  code boundary
//   k_decode       the table decode for codes of up to 64 bits
#include <hip/hip_runtime.h>

#include <type_traits>

#include "hc_internal.h"
#include "hc_kernels.h"

// Global address space.  Buffer pointers read from a job descriptor are
// otherwise generic, and generic (flat) loads also count against the LDS wait
// counter, which would make every LDS wait also wait for in-flight HBM loads.
#define HC_G __attribute__((address_space(1)))

typedef uint32_t v4u __attribute__((ext_vector_type(4)));  // 16-byte global loads/stores
typedef uint32_t v2u __attribute__((ext_vector_type(2)));

namespace hc {

// ---------------------------------------------------------------- helpers
// Streaming accesses marked non-temporal (kept out of the caches' reuse
// sets).  On MI355X this lifts a plain streaming copy from about 5.7 to
// 6.2 TB/s, but within the codec it pays only in the histogram's input reads
// (0.79 -> 0.67 ms over 4 GiB): the length pass, the packing and the copy
// forms ran slower with it, the staged decoder no faster.
template <typename T>
__device__ __forceinline__ T ld_nt(const HC_G T *p)
{
    return __builtin_nontemporal_load(p);
}

__device__ __forceinline__ void report(uint32_t *err, uint32_t code)
{
    // the plain read first: once the word holds an error, the many lanes of a
    // corrupt stream do not all queue on one atomic
    if (err && *(volatile uint32_t *)err == 0u) atomicCAS(err, 0u, code);
}

// Inclusive scan of 32-bit values over the 64 lanes with data-parallel moves
// (DPP), every lane active: within each row of 16 lanes by shifts of 1, 2, 4
// and 8, then the total of row 0 into row 1 and of row 2 into row 3 (lane 15's
// broadcast), then that of rows 0-1 into rows 2-3 (lane 31's).  Each step is
// a VALU move, where a lane exchange through the LDS unit waits on a round
// trip.  Op: + or |, identity 0 (a lane with no source in range adds 0).
template <bool kOr>
__device__ __forceinline__ uint32_t wave_scan_dpp(uint32_t x)
{
    auto step = [&](auto ctrl, auto rows) {
        const uint32_t y =
            __builtin_amdgcn_update_dpp(0u, x, decltype(ctrl)::value, decltype(rows)::value, 0xF, false);
        x = kOr ? (x | y) : (x + y);
    };
    using std::integral_constant;
    step(integral_constant<int, 0x111>(), integral_constant<int, 0xF>());  // row_shr:1
    step(integral_constant<int, 0x112>(), integral_constant<int, 0xF>());  // row_shr:2
    step(integral_constant<int, 0x114>(), integral_constant<int, 0xF>());  // row_shr:4
    step(integral_constant<int, 0x118>(), integral_constant<int, 0xF>());  // row_shr:8
    step(integral_constant<int, 0x142>(), integral_constant<int, 0xA>());  // row_bcast:15 into rows 1, 3
    step(integral_constant<int, 0x143>(), integral_constant<int, 0xC>());  // row_bcast:31 into rows 2, 3
    return x;
}

// Every caller runs it with all 64 lanes of the wave active.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x)
{
    if constexpr (std::is_same<T, uint32_t>::value) {
        return wave_scan_dpp<false>(x);
    } else {
        const int lane = threadIdx.x & 63;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            T y = __shfl_up(x, d, 64);
            if (lane >= d) x += y;
        }
        return x;
    }
}

// Every caller runs it with all 64 lanes of the wave active.
template <typename T>
__device__ __forceinline__ T wave_sum(T x)
{
    if constexpr (std::is_same<T, uint32_t>::value)
        return (uint32_t)__builtin_amdgcn_readlane(wave_scan_dpp<false>(x), 63);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

// Lane 'l''s 64-bit value in every lane, as a scalar.  The lane read
// returns a signed int: each half is taken as uint32_t before widening, or
// the low half would be sign-extended into the high one.
__device__ __forceinline__ uint64_t read_lane_u64(uint64_t v, int l)
{
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((uint32_t)(v >> 32), l);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((uint32_t)v, l);
    return ((uint64_t)hi << 32) | lo;
}

// Exclusive scan across the work-group; 'scratch' holds one entry per wave.
// Contains two barriers; every thread of the group must call it.
template <typename T, int NT>
__device__ __forceinline__ T group_exclusive_scan(T v, T *scratch, T *total)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    T inc = wave_inclusive_scan(v);
    if (lane == 63) scratch[wave] = inc;
    __syncthreads();
    T before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        T s = scratch[w];
        before += (w < wave) ? s : T(0);
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

__global__ void k_fill_u64(uint64_t *p, uint64_t count, uint64_t value)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// Up to kJobsPerPut jobs of a table travel by value as one launch's arguments.
constexpr uint32_t kJobsPerPut = 32;
struct JobChunk {
    Job jobs[kJobsPerPut];
    uint32_t first, count;  // table entries [first, first + count)
    uint32_t table_count;   // entries of the whole table
    uint64_t total;         // units of the whole table, after the last start
};

__global__ void k_put_jobs(JobChunk c, Job *jobs, uint64_t *starts)
{
    const uint32_t t = threadIdx.x;
    if (t < c.count) {
        jobs[c.first + t] = c.jobs[t];
        starts[c.first + t] = c.jobs[t].unit_begin;
    }
    if (t == 0 && c.first + c.count == c.table_count) starts[c.table_count] = c.total;
}

// The job owning launch unit u (the last job whose unit_begin <= u), found by
// the 64 lanes of one wave together: each round samples 64 job starts and
// keeps the bracket of the last one <= u, so 10^4 jobs take 3 rounds of one
// coalesced load.  Called by every lane of the wave; all lanes return it.
__device__ uint32_t wave_job_of_unit(const JobList &jl, uint64_t u)
{
    if (jl.count == 1) return 0;
    const uint32_t lane = threadIdx.x & 63;
    const HC_G uint64_t *starts = (const HC_G uint64_t *)jl.starts;
    uint32_t lo = 0, hi = jl.count;  // starts[lo] <= u always holds
    while (hi - lo > 1) {
        const uint32_t stride = (hi - lo + 63) / 64;
        const uint32_t k = lo + lane * stride;
        const uint64_t le = __ballot(k < hi && starts[k] <= u);
        lo += (63 - (uint32_t)__clzll((long long)le)) * stride;
        hi = lo + stride < hi ? lo + stride : hi;
    }
    return lo;
}

__device__ __forceinline__ Job job_at(const JobList &jl, uint32_t k) { return jl.jobs ? jl.jobs[k] : jl.one; }

// ---------------------------------------------------------------- histogram
// Each work-group counts a contiguous chunk into 64 LDS sub-histograms laid
// out bin-major (sub-histogram r of bin v at v*64 + r); lane r of every wave
// adds into sub-histogram r, so the 64 lanes of one LDS atomic always touch 64
// consecutive words whatever the data (no bank conflicts, no same-address
// serialisation on skewed inputs).  The group then folds the 64 copies and adds
// its counts to the global u64 histogram.
__global__ void k_hist_zero(JobList jl)
{
    const Job jb = job_at(jl, blockIdx.x);
    if (threadIdx.x < (uint32_t)kNumSym) jb.hist[threadIdx.x] = 0;
}

__global__ __launch_bounds__(kHistThreads) void k_hist(JobList jl, uint64_t chunk)
{
    __shared__ uint32_t sh[kNumSym * 64];
    __shared__ Job s_job;
    if (threadIdx.x < 64) {
        const uint32_t k = wave_job_of_unit(jl, blockIdx.x);
        if (threadIdx.x == 0) s_job = job_at(jl, k);
    }
    for (int k = threadIdx.x; k < kNumSym * 64; k += kHistThreads) sh[k] = 0;
    __syncthreads();

    const HC_G uint8_t *__restrict__ in = (const HC_G uint8_t *)s_job.in;
    const uint64_t n = s_job.n;
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t beg = (blockIdx.x - s_job.unit_begin) * chunk;
    const uint64_t end = beg + chunk < n ? beg + chunk : n;
    const uint64_t nvec = (end - beg) >> 4;
    const HC_G v4u *p = (const HC_G v4u *)(in + beg);

    auto add_word = [&](uint32_t w) {
        atomicAdd(&sh[((w)&255u) * 64 + lane], 1u);
        atomicAdd(&sh[((w >> 8) & 255u) * 64 + lane], 1u);
        atomicAdd(&sh[((w >> 16) & 255u) * 64 + lane], 1u);
        atomicAdd(&sh[(w >> 24) * 64 + lane], 1u);
    };
    auto add_vec = [&](v4u q) {
        add_word(q.x);
        add_word(q.y);
        add_word(q.z);
        add_word(q.w);
    };

    uint64_t v = threadIdx.x;
    for (; v + 3 * kHistThreads < nvec; v += 4 * kHistThreads) {
        v4u a = ld_nt(p + v);
        v4u b = ld_nt(p + v + kHistThreads);
        v4u c = ld_nt(p + v + 2 * kHistThreads);
        v4u d = ld_nt(p + v + 3 * kHistThreads);
        add_vec(a);
        add_vec(b);
        add_vec(c);
        add_vec(d);
    }
    for (; v < nvec; v += kHistThreads) add_vec(ld_nt(p + v));
    for (uint64_t j = beg + (nvec << 4) + threadIdx.x; j < end; j += kHistThreads)
        atomicAdd(&sh[(uint32_t)in[j] * 64 + lane], 1u);
    __syncthreads();

    if (threadIdx.x < kNumSym) {
        const uint32_t b = threadIdx.x;
        uint64_t s = 0;
#pragma unroll 8
        for (uint32_t r = 0; r < 64; ++r) s += sh[b * 64 + ((r + b) & 63u)];  // rotated: no conflicts
        if (s) atomicAdd(reinterpret_cast<unsigned long long *>(&s_job.hist[b]), (unsigned long long)s);
    }
}

// ---------------------------------------------------------------- tiles
__device__ __forceinline__ uint64_t num_blocks_dev(uint64_t n, uint32_t B) { return (n + B - 1) / B; }

struct Tile {
    uint64_t blk;       // block index
    uint32_t j;         // tile index inside the block
    uint64_t blk_start; // first symbol of the block
    uint32_t cnt;       // symbols in the block
    uint32_t ts, te;    // symbol range of the tile, relative to the block
};

// Tile t (counted from the job's first tile) of a job of n symbols: tiles of
// tile_syms symbols, tpb of them per block.
__device__ __forceinline__ Tile tile_of(uint64_t n, uint32_t B, uint32_t tpb, uint32_t tile_syms, uint64_t t)
{
    Tile r;
    r.blk = t / tpb;
    r.j = (uint32_t)(t - r.blk * tpb);
    r.blk_start = r.blk * (uint64_t)B;
    const uint64_t left = n - r.blk_start;
    r.cnt = (uint32_t)(left < B ? left : B);
    r.ts = r.j * tile_syms;
    const uint32_t e = r.ts + tile_syms;
    r.te = e < r.cnt ? e : r.cnt;
    if (r.ts > r.te) r.ts = r.te;  // empty tile past the end of a short last block
    return r;
}

// Loads the (up to) 16*QPT consecutive symbols of this thread from symbol s
// of the tile's block; returns how many there are.
template <uint32_t QPT>
__device__ __forceinline__ uint32_t load_syms(const HC_G uint8_t *__restrict__ in, const Tile &tl, uint32_t s,
                                              uint32_t w[4 * QPT])
{
#pragma unroll
    for (uint32_t i = 0; i < 4 * QPT; ++i) w[i] = 0;
    if (s >= tl.te) return 0;
    const HC_G uint8_t *src = in + tl.blk_start + s;
    if (s + kQuadSyms * QPT <= tl.te) {
#pragma unroll
        for (uint32_t q = 0; q < QPT; ++q) {
            const v4u v = ((const HC_G v4u *)src)[q];
            w[4 * q + 0] = v.x;
            w[4 * q + 1] = v.y;
            w[4 * q + 2] = v.z;
            w[4 * q + 3] = v.w;
        }
        return kQuadSyms * QPT;
    }
    // the ragged end of a block: whole words, then the bytes of a last partial word
    const uint32_t m = tl.te - s;
    const uint32_t full = m >> 2;
    const HC_G uint32_t *src32 = (const HC_G uint32_t *)src;
#pragma unroll
    for (uint32_t i = 0; i < 4 * QPT; ++i)
        if (i < full) w[i] = src32[i];
    uint32_t part = 0;
    for (uint32_t b = 0; b < (m & 3u); ++b) part |= (uint32_t)src[4 * full + b] << (8 * b);
#pragma unroll
    for (uint32_t i = 0; i < 4 * QPT; ++i)
        if (i == full && (m & 3u)) w[i] = part;
    return m;
}

__device__ __forceinline__ uint32_t sym_at(const uint32_t w[4], uint32_t k)
{
    return (w[k >> 2] >> (8 * (k & 3))) & 255u;
}

// ---------------------------------------------------------------- pack
// Appends the low L bits of 'code' (L <= 32) to a thread's bit accumulator and
// flushes every completed 32-bit word into LDS.
__device__ __forceinline__ void put_bits(uint64_t &acc, uint32_t &nacc, uint32_t &widx, uint32_t code,
                                         uint32_t L, uint32_t *words)
{
    acc = (acc << L) | code;
    nacc += L;
    if (nacc >= 32) {
        nacc -= 32;
        atomicOr(&words[widx++], (uint32_t)(acc >> nacc));
        acc &= (nacc ? ((1ull << nacc) - 1) : 0ull);
    }
}

// ---------------------------------------------------------------- encode
// Three launches, in the paper's order (section 2.1): the length pass counts
// the bits of every tile, the offset pass turns them into the position of
// every tile inside its block and the byte offset of every block, and the
// packing pass writes each tile's code words there.  No launch waits on
// another work-group, so every work-group runs from start to end at once.

// Length pass: work-group t sums the code lengths of tile t (the same tile
// shape as the packing pass) and reports a symbol without a code.  The
// lengths come from 64 LDS replicas of the table, four lengths per word, and
// lane r reads replica r (word i at [64 i + r]): a wave's 64 lookups then
// hit 64 distinct banks whatever the symbols, where one shared table makes
// uniform data conflict several ways per lookup.  With thread_bits, each
// thread's own sum is kept for the packing pass too.  Built for 8 waves per
// SIMD, as the packing pass.
template <uint32_t QPT>
__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_count(JobList jl, uint32_t B, uint32_t tpb, uint32_t *tile_bits,
                                                        uint16_t *thread_bits, uint32_t shape_len, uint32_t *err)
{
    constexpr uint32_t kSyms = kQuadSyms * QPT;
    constexpr uint32_t kWords = kNumSym / 4;  // length words per replica
    __shared__ __attribute__((aligned(16))) uint32_t s_len4[64 * kWords];
    __shared__ uint32_t s_red[kTileThreads / 64];
    __shared__ Job s_job;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const uint64_t t = blockIdx.x;
    if (tid < 64) {
        const uint32_t k = wave_job_of_unit(jl, t);
        if (tid == 0) s_job = job_at(jl, k);
    }
    __syncthreads();
    const HC_G DevTables *__restrict__ tb = (const HC_G DevTables *)s_job.tb;
    const HC_G uint8_t *__restrict__ in = (const HC_G uint8_t *)s_job.in;
    const Tile tl = tile_of(s_job.n, B, tpb, kTileSyms * QPT, t - s_job.unit_begin);
    const uint32_t s = tl.ts + kSyms * tid;
    // The input and the length words are requested before the table is
    // checked, so that their latency overlaps the check's reads instead of
    // following them (a group's whole life is a few of these latencies).
    uint32_t w[4 * QPT];
    const uint32_t m = load_syms<QPT>(in, tl, s, w);  // 0 past the end of the tile
    const v4u x = ((const HC_G v4u *)tb->len4)[tid >> 4];
    if (tb->max_len > shape_len) {  // the same in every lane: the group leaves together
        // (the loads' results are named on this path too, so that they stay
        // ahead of the check rather than being sunk past it)
        asm volatile("" ::"v"(w[0]), "v"(x.x));
        if (tid == 0) report(err, HC_ERR_TABLE_CHANGED);
        return;
    }
    if (tb->fixed_len == 8 && tb->count[8] == (uint32_t)kNumSym) {
        // A complete 8-bit code (uniform over the group: one job per tile):
        // every symbol has a code of 8 bits, so the count needs no input; the
        // packing pass copies such tiles without per-thread counts.  (Launches
        // are shaped so that such codes run no length pass at all.)
        if (tid == 0) tile_bits[t] = tl.ts < tl.te ? 8 * (tl.te - tl.ts) : 0u;
        return;
    }
    {
        // thread t holds words 4q..4q+3 (q = t / 16) and writes each into
        // replicas 4g..4g+3 (g = t mod 16): one 16-byte load, four 16-byte LDS
        // writes, and each write instruction covers all banks evenly
        static_assert(kWords == 64 && kTileThreads == 256, "one length word group per 16 threads");
        const uint32_t q = tid >> 4, g = tid & 15u;
        const uint32_t xs[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j)
            *(v4u *)(s_len4 + 64 * (4 * q + j) + 4 * g) = v4u{xs[j], xs[j], xs[j], xs[j]};
    }
    __syncthreads();
    // Symbol v's length is byte 256 (v >> 2) + 4 lane + (v & 3) of the
    // replicas: one byte read, its address one byte permute per symbol from two
    // words made once per four symbols, (v >> 2) in each byte of one and
    // 4 lane + (v & 3) in each byte of the other.  The length pass is bound by
    // VALU issue, and this takes the per-symbol address and extract work from
    // six instructions to one.
    const uint8_t *len8 = (const uint8_t *)s_len4;
    const uint32_t lane4 = (lane * 4u) * 0x01010101u;
    uint32_t bits = 0, mn = 255u;  // mn: the smallest code length met, 0 = a symbol without a code
    // Only the wave holding a block's ragged end masks symbols past m.
    auto count = [&](auto mask_tag) {
        constexpr bool kMask = decltype(mask_tag)::value;
#pragma unroll
        for (uint32_t i = 0; i < 4 * QPT; ++i) {
            if ((i & 3u) == 0 && i) {
                // one load's lookups at a time: bounds the registers held by reads in flight
                __builtin_amdgcn_sched_barrier(0);
                asm volatile("" : "+v"(w[i]), "+v"(w[i + 1]), "+v"(w[i + 2]), "+v"(w[i + 3]), "+v"(bits), "+v"(mn));
            }
            const uint32_t hi = (w[i] >> 2) & 0x3F3F3F3Fu;
            const uint32_t lo = (w[i] & 0x03030303u) | lane4;
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) {
                const uint32_t k = 4 * i + j;
                // byte 0 <- byte j of lo, byte 1 <- byte j of hi, bytes 2-3 <- 0
                const uint32_t a = __builtin_amdgcn_perm(hi, lo, 0x0C0C0000u | ((4u + j) << 8) | j);
                const uint32_t L = len8[a];
                bits += (!kMask || k < m) ? L : 0u;
                mn = min(mn, (!kMask || k < m) ? L : 255u);
            }
        }
    };
    if (__all(m == kSyms))
        count(std::integral_constant<bool, false>());
    else
        count(std::integral_constant<bool, true>());
    if (mn == 0) report(err, HC_ERR_SYMBOL_ABSENT);
    if (thread_bits) thread_bits[t * kTileThreads + tid] = (uint16_t)bits;  // <= 64 codes of <= 24 bits
    bits = wave_sum(bits);
    if (lane == 0) s_red[wave] = bits;
    __syncthreads();
    if (tid == 0) {
        uint32_t total = 0;
#pragma unroll
        for (int wv = 0; wv < kTileThreads / 64; ++wv) total += s_red[wv];
        tile_bits[t] = total;
    }
}

// Offset pass: work-group k scans job k.  Each thread takes kOffBlocks
// consecutive blocks per round: the exclusive sums of their tiles' bit counts
// are the tiles' positions inside the block, the block's size is a 4-byte
// header plus its payload padded to whole 32-bit words, and a group scan of
// the threads' byte totals gives every block's offset (the last entry of the
// table is the stream size).
constexpr uint32_t kOffThreads = 256;
constexpr uint32_t kOffBlocks = 16;

// c8_tile_syms > 0: every job of the launch has a complete 8-bit code and
// tiles of c8_tile_syms symbols, so a tile's bit count is 8 times its
// symbols and no length pass ran (a job whose table no longer has such a
// code reports TABLE_CHANGED).
__global__ __launch_bounds__(kOffThreads) void k_offsets(JobList jl, uint32_t B, uint32_t tpb,
                                                         const uint32_t *tile_bits, uint32_t *tile_pos,
                                                         uint32_t c8_tile_syms, uint32_t *err)
{
    __shared__ uint64_t s_scan[kOffThreads / 64];
    const Job jb = job_at(jl, blockIdx.x);
    if (jb.n == 0) return;  // the empty stream's table is written on its own
    const uint32_t tid = threadIdx.x;
    if (c8_tile_syms) {
        const HC_G DevTables *__restrict__ tb = (const HC_G DevTables *)jb.tb;
        if (!(tb->fixed_len == 8 && tb->count[8] == (uint32_t)kNumSym)) {  // the same in every lane
            if (tid == 0) report(err, HC_ERR_TABLE_CHANGED);
            return;
        }
    }
    const uint64_t nb = num_blocks_dev(jb.n, B);
    const HC_G uint32_t *tbits = (const HC_G uint32_t *)tile_bits + jb.unit_begin;
    HC_G uint32_t *tpos = (HC_G uint32_t *)tile_pos + jb.unit_begin;
    HC_G uint64_t *block_off = (HC_G uint64_t *)jb.block_off;
    uint64_t carry = 0;
    for (uint64_t b0 = 0; b0 < nb; b0 += (uint64_t)kOffThreads * kOffBlocks) {
        const uint64_t first = b0 + (uint64_t)tid * kOffBlocks;
        uint32_t bytes[kOffBlocks];
        uint64_t mine = 0;
#pragma unroll
        for (uint32_t i = 0; i < kOffBlocks; ++i) {
            const uint64_t b = first + i;
            bytes[i] = 0;
            if (b < nb) {
                uint64_t bits = 0;
                if (c8_tile_syms) {
                    const uint64_t left = jb.n - b * (uint64_t)B;
                    const uint32_t cnt = (uint32_t)(left < B ? left : B);
                    for (uint32_t j = 0; j < tpb; ++j) {
                        tpos[b * tpb + j] = (uint32_t)bits;
                        const uint32_t ts = j * c8_tile_syms;
                        bits += ts < cnt ? 8ull * (cnt - ts < c8_tile_syms ? cnt - ts : c8_tile_syms) : 0ull;
                    }
                } else {
                    for (uint32_t j = 0; j < tpb; ++j) {
                        tpos[b * tpb + j] = (uint32_t)bits;
                        bits += tbits[b * tpb + j];
                    }
                }
                if (bits > 0xFFFFFFFFull) report(err, HC_ERR_BLOCK_OVERFLOW);
                bytes[i] = (uint32_t)(4 + 4 * ((bits + 31) / 32));
                mine += bytes[i];
            }
        }
        uint64_t total;
        uint64_t off = carry + group_exclusive_scan<uint64_t, kOffThreads>(mine, s_scan, &total);
#pragma unroll
        for (uint32_t i = 0; i < kOffBlocks; ++i) {
            if (first + i < nb) block_off[first + i] = off;
            off += bytes[i];
        }
        carry += total;
    }
    if (tid == 0) block_off[nb] = carry;
}

// kPacked: codes of <= 24 bits from the packed table, FPS codes between
// accumulator flushes (FPS * max_len <= 32); otherwise codes up to 64 bits.
// QPT: 16-symbol loads per thread; a tile is 4096 * QPT symbols and thread i
// codes its symbols [16 * QPT * i, 16 * QPT * (i + 1)).  With QPT >= 2 the
// length pass has kept every thread's bit count (thread_bits), so each symbol
// is looked up once here; tiles of 4096 symbols count their bits again
// rather than move a count per 16 symbols through HBM.
// Built for 8 waves per SIMD (<= 64 VGPRs): 8 work-groups per CU in flight.
template <bool kPacked, uint32_t FPS, uint32_t QPT>
__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_encode(
    JobList jl, uint32_t B, uint32_t tpb, const uint32_t *tile_pos, const uint16_t *thread_bits, uint32_t S,
    uint32_t cpb, uint32_t lds_words, uint32_t shape_len, uint32_t copy_only, uint32_t *err)
{
    constexpr uint32_t kSyms = kQuadSyms * QPT;  // symbols per thread
    constexpr bool kHanded = QPT >= 2;           // bit counts from the length pass
    static_assert(!kHanded || kPacked, "tiles of more than 4096 symbols hold codes of <= 24 bits");
    extern __shared__ __attribute__((aligned(16))) uint32_t words[];  // the tile's code bits from bit 0, MSB first
    __shared__ uint32_t s_packed[kNumSym];
    __shared__ uint64_t s_code[kPacked ? 1 : kNumSym];
    __shared__ uint32_t s_len[kPacked ? 1 : kNumSym];
    __shared__ uint32_t s_scan[kTileThreads / 64];
    __shared__ uint32_t s_lead;
    __shared__ uint32_t s_next[32];  // the first symbols of the next tile of the block
    __shared__ uint64_t s_P, s_O;
    __shared__ Job s_job;

    const uint32_t tid = threadIdx.x;
    const uint64_t t = blockIdx.x;
    if (tid < 64) {
        const uint32_t k = wave_job_of_unit(jl, t);
        if (tid == 0) s_job = job_at(jl, k);
    }
    __syncthreads();
    const HC_G DevTables *__restrict__ tb = (const HC_G DevTables *)s_job.tb;
    const HC_G uint8_t *__restrict__ in = (const HC_G uint8_t *)s_job.in;
    HC_G uint32_t *__restrict__ out32 = (HC_G uint32_t *)s_job.out;
    HC_G uint32_t *__restrict__ sub_idx = (HC_G uint32_t *)s_job.sub_idx;
    const Tile tl = tile_of(s_job.n, B, tpb, kTileSyms * QPT, t - s_job.unit_begin);
    // The thread's symbols and bit count are requested before the table is
    // checked, so that their latency overlaps the check's reads instead of
    // following them.  Launches for complete 8-bit codes copy the tile
    // instead and request nothing here.
    const uint32_t s = tl.ts + kSyms * tid;
    uint32_t w[4 * QPT];
#pragma unroll
    for (uint32_t i = 0; i < 4 * QPT; ++i) w[i] = 0;
    uint32_t m = copy_only ? 0u : load_syms<QPT>(in, tl, s, w);
    uint32_t bits = (kHanded && !copy_only) ? (uint32_t)thread_bits[t * kTileThreads + tid] : 0u;
    const uint32_t packed = kPacked ? tb->enc_packed[tid] : 0u;
    if (tb->max_len > shape_len) {  // the same in every lane: the group leaves together
        // (the loads' results are named on this path too, so that they stay
        // ahead of the check rather than being sunk past it)
        asm volatile("" ::"v"(w[0]), "v"(bits), "v"(packed));
        if (tid == 0) report(err, HC_ERR_TABLE_CHANGED);
        return;
    }
    if (kPacked) {
        s_packed[tid] = packed;
    } else {
        s_code[tid] = tb->enc_code[tid];
        s_len[tid] = tb->enc_len[tid];
    }
    if (tl.ts >= tl.te) return;  // empty tile past a short last block (uniform over the group)

    const bool last_tile = tl.te == tl.cnt;
    const bool c8 = tb->fixed_len == 8 && tb->count[8] == (uint32_t)kNumSym;
    if (copy_only && !c8) {  // a launch shaped for complete 8-bit codes only (no length pass ran)
        if (tid == 0) report(err, HC_ERR_TABLE_CHANGED);
        return;
    }
    if (c8) {
        // A complete 8-bit code (uniform over the group): every symbol is its
        // own code, a tile starts on a whole word (P is 8 times a multiple of
        // 4096) and shares no word with the next tile, so the tile's payload
        // is its input words byte-swapped (the first symbol into a word's top
        // byte), copied with thread k on word k (coalesced both ways).  A
        // last partial word is assembled from bytes; its missing bytes are
        // the zero pad.
        const uint64_t P = tile_pos[t], O = ((const HC_G uint64_t *)s_job.block_off)[tl.blk];
        HC_G uint32_t *payload = out32 + (O >> 2) + 1 + (P >> 5);
        const HC_G uint8_t *src8 = in + tl.blk_start + tl.ts;  // 16-byte aligned: B and the tile are multiples of 16
        const HC_G uint32_t *src = (const HC_G uint32_t *)src8;
        const uint32_t nsym = tl.te - tl.ts, nfull = nsym / 4, nvec = nsym / 16;
        // 16-byte pieces, four in flight per thread (a tile of 4096 * QPT
        // symbols is QPT rounds); each piece's four words go to the payload,
        // which sits on any word (so a thread's words are four stores, the
        // wave's stores covering a contiguous 1 KiB together)
        for (uint32_t v0 = 0; v0 < nvec; v0 += 4 * kTileThreads) {
            v4u x[4];
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u) {
                const uint32_t v = v0 + u * kTileThreads + tid;
                if (v < nvec) x[u] = ((const HC_G v4u *)src8)[v];
            }
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u) {
                const uint32_t v = v0 + u * kTileThreads + tid;
                if (v < nvec) {
                    HC_G uint32_t *d = payload + 4 * v;
                    d[0] = __builtin_bswap32(x[u].x);
                    d[1] = __builtin_bswap32(x[u].y);
                    d[2] = __builtin_bswap32(x[u].z);
                    d[3] = __builtin_bswap32(x[u].w);
                }
            }
        }
        if (tid < nfull - 4 * nvec) payload[4 * nvec + tid] = __builtin_bswap32(src[4 * nvec + tid]);  // < 4 whole words
        if ((nsym & 3) && tid == 0) {
            uint32_t part = 0;
            for (uint32_t b = 0; b < (nsym & 3); ++b) part |= (uint32_t)src8[4 * nfull + b] << (8 * b);
            payload[nfull] = __builtin_bswap32(part);
        }
        const uint32_t blk_bits = (uint32_t)P + 8 * nsym;
        if (last_tile && tid == 0) out32[O >> 2] = blk_bits;
        if (sub_idx) {
            // entries at the multiples of S in the tile, 8 bits per symbol
            for (uint32_t sj = tl.ts + (S - tl.ts % S) % S + tid * S; sj < tl.te; sj += kTileThreads * S)
                sub_idx[tl.blk * cpb + sj / S] = (uint32_t)P + 8 * (sj - tl.ts);
            if (last_tile && tid == 0)
                for (uint32_t c = (tl.cnt + S - 1) / S; c < cpb; ++c) sub_idx[tl.blk * cpb + c] = blk_bits;
        }
        return;
    }
    // the tile's words start at zero (ordered before the packing's ors by the
    // barrier below), 16 bytes per write: lds_words is a multiple of 4
    for (uint32_t k = 4 * tid; k < lds_words; k += 4 * kTileThreads) *(v4u *)(words + k) = v4u{0u, 0u, 0u, 0u};
    const uint32_t avail = last_tile ? 0u : (tl.cnt - tl.te < 32 ? tl.cnt - tl.te : 32u);
    if (tid < 32) s_next[tid] = tid < avail ? in[tl.blk_start + tl.te + tid] : 0u;
    if (tid == 32) {  // where the tile's bits go: from the offset pass
        s_P = tile_pos[t];
        s_O = ((const HC_G uint64_t *)s_job.block_off)[tl.blk];
    }
    __syncthreads();  // code tables and the next tile's first symbols are in LDS

    // Without handed counts the thread's symbols are coded twice from the LDS
    // table: once for their bit count (before the group scan), once to pack
    // them (after it).  Holding 16*QPT table entries per thread across the
    // scan would cost more registers than the second reads cost time.  Waves
    // whose threads all hold full loads take the variant without per-symbol
    // masks (kMask false); only the wave with the ragged end of a block needs
    // them (symbols past m then read entry 0 and are masked to zero).
    const bool wave_full = __all(m == kSyms);
    uint32_t qbits[QPT];  // the thread's bits before each of its loads (sub-block index)
    auto count_bits = [&](auto mask_tag) {
        constexpr bool kMask = decltype(mask_tag)::value;
        uint32_t mn = 255u;  // the smallest code length met: 0 = a symbol without a code
#pragma unroll
        for (uint32_t k = 0; k < kSyms; ++k) {
            if ((k & (kQuadSyms - 1)) == 0) {
                // one load's lookups at a time: bounds the registers held by reads in flight
                if (k) __builtin_amdgcn_sched_barrier(0);
                const uint32_t i = k / 4;  // this load's words become opaque here: no early address math
                asm volatile("" : "+v"(w[i]), "+v"(w[i + 1]), "+v"(w[i + 2]), "+v"(w[i + 3]), "+v"(bits));
                qbits[k / kQuadSyms] = bits;
            }
            const uint32_t e = kPacked ? (s_packed[sym_at(w, k)] & 255u) : s_len[sym_at(w, k)];
            const uint32_t L = (!kMask || k < m) ? e : 0u;
            mn = min(mn, (!kMask || k < m) ? e : 255u);
            bits += L;
        }
        if (mn == 0) report(err, HC_ERR_SYMBOL_ABSENT);
    };
    if (kHanded)
        ;
    else if (wave_full)
        count_bits(std::integral_constant<bool, false>());
    else
        count_bits(std::integral_constant<bool, true>());
    uint32_t tile_total;
    const uint32_t q = group_exclusive_scan<uint32_t, kTileThreads>(bits, s_scan, &tile_total);

    {  // pack at alignment 0
        asm volatile("" : "+v"(m) : : "memory");  // table reads and (k < m) masks are redone
        uint32_t widx = q >> 5;
        uint32_t nacc = q & 31u;  // leading zero bits keep the word aligned
        uint64_t acc = 0;
        if (kPacked) {
            // FPS codes of <= 32/FPS bits are first joined in a 32-bit group
            // code (the entry's low 5 bits are the length, so one shift-or per
            // code), then appended to the accumulator, whose pending bits never
            // exceed 63; one flush retires at most one word.  The bits above
            // the pending ones are left in place, not cleared: every word taken
            // out of the accumulator is 32 bits ending at its last pending bit,
            // so they never reach one.
            const uint32_t pos0 = q;  // the thread's first bit in the tile
            auto pack = [&](auto mask_tag) {
                constexpr bool kMask = decltype(mask_tag)::value;
                // groups of FPS codes inside each 16-symbol load (FPS = 3
                // leaves a last group of one), so that a load's first symbol
                // always starts a group (the sub-block index positions)
                constexpr uint32_t kGroups = (kQuadSyms + FPS - 1) / FPS;
#pragma unroll
                for (uint32_t q = 0; q < QPT; ++q) {
                    if (q) __builtin_amdgcn_sched_barrier(0);
                    asm volatile("" : "+v"(w[4 * q]), "+v"(w[4 * q + 1]), "+v"(w[4 * q + 2]), "+v"(w[4 * q + 3]));
                    if (kHanded) qbits[q] = 32 * widx + nacc - pos0;  // the thread's bits so far
#pragma unroll
                    for (uint32_t g = 0; g < kGroups; ++g) {
                        const uint32_t k = kQuadSyms * q + FPS * g;
                        const uint32_t G = g + 1 < kGroups ? FPS : kQuadSyms - FPS * g;  // codes in this group
                        uint32_t gc = 0, gsum = 0;
#pragma unroll
                        for (uint32_t j = 0; j < FPS; ++j) {
                            if (j < G) {
                                const uint32_t e0 = s_packed[sym_at(w, k + j)];
                                const uint32_t e = (!kMask || k + j < m) ? e0 : 0u;
                                gc = (gc << (e & 31u)) | (e >> 8);
                                gsum += e;  // the low byte sums the lengths (<= 32)
                            }
                        }
                        // gsum's low byte is the group's length (<= 32); what
                        // it holds above that only reaches bits >= 8 of nacc,
                        // which the flush clears before they are read
                        acc = (acc << (gsum & 63u)) | gc;
                        nacc += gsum;
                        // bit 5 of nacc: a whole word is pending (nacc <= 63);
                        // it is the 32 bits ending at the last pending bit
                        const uint32_t full = (uint32_t)((int32_t)(nacc << 26) >> 31);  // all ones or zero
                        const uint32_t word = __builtin_amdgcn_alignbit((uint32_t)(acc >> 32), (uint32_t)acc, nacc);
                        atomicOr(&words[widx], word & full);
                        widx -= full;  // one word on when one was retired
                        nacc &= 31u;
                    }
                }
            };
            if (wave_full)
                pack(std::integral_constant<bool, false>());
            else
                pack(std::integral_constant<bool, true>());
        } else {
#pragma unroll
            for (uint32_t k = 0; k < kSyms; ++k) {
                if (k < m) {
                    const uint32_t v = sym_at(w, k);
                    const uint32_t L = s_len[v];
                    const uint64_t c = s_code[v];
                    if (L > 32) {
                        put_bits(acc, nacc, widx, (uint32_t)(c >> 32), L - 32, words);
                        put_bits(acc, nacc, widx, (uint32_t)c, 32, words);
                    } else {
                        put_bits(acc, nacc, widx, (uint32_t)c, L, words);
                    }
                }
            }
        }
        if (nacc) atomicOr(&words[widx], (uint32_t)(acc << (32 - nacc)));
    }

    // The first 32 bits of the next tile of the block (zero past the block's
    // end): they complete this tile's last stream word.
    if (kPacked) {
        if (tid >= 64 && tid < 128) {  // wave 1: one symbol per lane, placed by a scan of lengths
            const uint32_t l = tid - 64;
            const uint32_t e = (l < avail) ? s_packed[s_next[l]] : 0u;
            const uint32_t L = e & 255u;
            const uint32_t pos = wave_inclusive_scan(L) - L;
            // L <= 24: the code fits the 64-bit window when it starts in the first 32 bits
            const uint64_t v = (L && pos < 32) ? ((uint64_t)(e >> 8) << (64 - pos - L)) : 0ull;
            // the first 32 bits: the OR of every lane's high word (lane 63 holds it)
            const uint32_t lead = (uint32_t)__builtin_amdgcn_readlane(wave_scan_dpp<true>((uint32_t)(v >> 32)), 63);
            if (l == 0) s_lead = lead;
        }
    } else if (tid == 64) {
        uint64_t lead = 0;
        uint32_t got = 0;
        for (uint32_t k = 0; k < avail && got < 32; ++k) {
            const uint32_t v = s_next[k];
            const uint32_t L = s_len[v];
            const uint64_t c = s_code[v];
            const uint32_t r = 32 - got;
            if (L >= r) {
                lead = (lead << r) | (c >> (L - r));
                got = 32;
            } else {
                lead = (lead << L) | c;
                got += L;
            }
        }
        s_lead = (uint32_t)(lead << (32 - got));
    }

    __syncthreads();
    const uint64_t P = s_P, O = s_O;
    const uint32_t a = (uint32_t)(P & 31);
    HC_G uint32_t *payload = out32 + (O >> 2) + 1 + (P >> 5);
    if (tile_total) {
        // stream word k of the tile holds tile bits [32k - a, 32k - a + 32); it is
        // written here if its first bit is this tile's (k >= 1 when a > 0)
        const uint32_t e_bits = a + tile_total;
        const uint32_t k_last = (e_bits - 1) >> 5;
        const uint32_t fill = (!last_tile && (e_bits & 31u)) ? (s_lead >> (e_bits & 31u)) : 0u;
        const uint32_t k0 = a ? 1u : 0u;  // word 0 is the previous tile's when a > 0
        auto word_at = [&](uint32_t k) { return a ? ((words[k - 1] << (32 - a)) | (words[k] >> a)) : words[k]; };
        // words k0 .. k_last - 1: four per thread per round, 256 apart, so
        // that each store instruction still writes 256 contiguous bytes while
        // the round's addresses are immediate offsets of one base
        const uint32_t nk = k_last > k0 ? k_last - k0 : 0u;
        if (a) {
            for (uint32_t g = tid; g < nk; g += 4 * kTileThreads) {
#pragma unroll
                for (uint32_t u = 0; u < 4; ++u) {
                    const uint32_t i = g + u * kTileThreads;  // stream word 1 + i
                    if (i < nk) payload[1 + i] = __builtin_amdgcn_alignbit(words[i], words[i + 1], a);
                }
            }
        } else {
            for (uint32_t g = tid; g < nk; g += 4 * kTileThreads) {
#pragma unroll
                for (uint32_t u = 0; u < 4; ++u) {
                    const uint32_t i = g + u * kTileThreads;
                    if (i < nk) payload[i] = words[i];
                }
            }
        }
        if (k_last >= k0 && tid == kTileThreads - 1) payload[k_last] = word_at(k_last) | fill;
    }
    const uint32_t blk_bits = (uint32_t)P + tile_total;  // the block's bit count, for its last tile
    if (last_tile && tid == 0) out32[O >> 2] = blk_bits;
    if (sub_idx) {
        // S and s are multiples of 16, so entries fall on the first symbol of
        // a load: e is the first entry at or after symbol s, 'at' its offset
        // from s, and each load's start is compared with it (one division
        // per thread rather than a remainder and a quotient per load)
        uint32_t e = (s + S - 1) / S, at = e * S - s;
#pragma unroll
        for (uint32_t j = 0; j < QPT; ++j) {
            if (m > kQuadSyms * j && at == kQuadSyms * j) {
                sub_idx[tl.blk * cpb + e] = (uint32_t)P + q + qbits[j];
                ++e;
                at += S;
            }
        }
        if (last_tile && tid == 0)
            for (uint32_t c = (tl.cnt + S - 1) / S; c < cpb; ++c) sub_idx[tl.blk * cpb + c] = blk_bits;
    }
}

// ---------------------------------------------------------------- walk
// The offset table from the length delimiters: each header gives the size of
// its block, so the walk is one dependent load per block (one lane).
__global__ void k_walk(const uint32_t *__restrict__ in32, uint64_t in_bytes, uint64_t nb,
                       uint64_t *__restrict__ off, uint32_t *err)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    uint64_t o = 0;
    off[0] = 0;
    for (uint64_t i = 0; i < nb; ++i) {
        if (o + 4 > in_bytes) {
            report(err, HC_ERR_CORRUPT);
            return;
        }
        const uint64_t bits = in32[o >> 2];
        o += 4 + 4 * ((bits + 31) / 32);
        if (o > in_bytes) {
            report(err, HC_ERR_CORRUPT);
            return;
        }
        off[i + 1] = o;
    }
    if (o != in_bytes) report(err, HC_ERR_CORRUPT);
}

// ---------------------------------------------------------------- decode
// The bit-reading helpers take the payload as global memory or as a copy in
// LDS (Ptr: a pointer to const u32 in either).
template <typename Ptr>
__device__ __forceinline__ uint32_t ld_word(Ptr payload, uint32_t nwords, uint32_t w)
{
    return w < nwords ? payload[w] : 0u;
}

// 64 payload bits starting at bit p (bits past the payload read as 0).
template <typename Ptr>
__device__ __forceinline__ uint64_t window64(Ptr payload, uint32_t nwords, uint64_t p)
{
    const uint32_t w = (uint32_t)(p >> 5), r = (uint32_t)(p & 31);
    uint64_t v = ((uint64_t)ld_word(payload, nwords, w) << 32) | ld_word(payload, nwords, w + 1);
    if (r) v = (v << r) | (ld_word(payload, nwords, w + 2) >> (32 - r));
    return v;
}

// Bit reader: 'buf' holds the next 'nbits' payload bits, most significant
// first; the bits after them start at word 'wi' (so the bit position is
// 32*wi - nbits at every step).
struct BitReader {
    uint64_t buf;
    uint32_t nbits;
    uint32_t wi;

    template <typename Ptr>
    __device__ __forceinline__ void seek(Ptr payload, uint32_t nwords, uint64_t p)
    {
        wi = (uint32_t)(p >> 5);
        const uint32_t r = (uint32_t)(p & 31);
        buf = (((uint64_t)ld_word(payload, nwords, wi) << 32) | ld_word(payload, nwords, wi + 1)) << r;
        nbits = 64 - r;
        wi += 2;
    }
    __device__ __forceinline__ uint64_t pos() const { return 32 * (uint64_t)wi - nbits; }
};

// Decodes one symbol.  Fast path: the next lut_bits bits index the LDS table.
// Codes longer than lut_bits are resolved by comparing the next 64 bits with
// the canonical code range of every longer length.
template <typename Ptr>
__device__ __forceinline__ uint32_t decode_one(BitReader &br, Ptr payload, uint32_t nwords, const uint16_t *lut,
                                               uint32_t K, uint32_t max_len, const uint64_t *first,
                                               const uint32_t *count, const uint32_t *base,
                                               const uint32_t *sorted, bool &bad)
{
    if (br.nbits < 32) {
        br.buf |= (uint64_t)ld_word(payload, nwords, br.wi) << (32 - br.nbits);
        br.nbits += 32;
        br.wi += 1;
    }
    const uint32_t e = lut[br.buf >> (64 - K)];
    const uint32_t L = e & 0x7Fu;
    if (e & kLutBadFlag) {  // no code starts with these bits
        bad = true;
        return 0;
    }
    if (L != 0) {
        br.buf <<= L;
        br.nbits -= L;
        return e >> 8;
    }
    const uint64_t p = br.pos();
    const uint64_t W = window64(payload, nwords, p);
    for (uint32_t l = K + 1; l <= max_len; ++l) {
        const uint64_t c = W >> (64 - l);
        const uint64_t d = c - first[l];
        if (d < count[l]) {
            br.seek(payload, nwords, p + l);
            return sorted[base[l] + (uint32_t)d];
        }
    }
    bad = true;
    return 0;
}

__global__ __launch_bounds__(kDecThreads) void k_decode(JobList jl, uint32_t B, uint32_t S_eff, uint32_t cpb,
                                                        uint32_t *err)
{
    __shared__ uint16_t s_lut[1 << kLutBits];
    __shared__ uint64_t s_first[kMaxLen + 1];
    __shared__ uint32_t s_count[kMaxLen + 1];
    __shared__ uint32_t s_base[kMaxLen + 1];
    __shared__ uint32_t s_sorted[kNumSym];
    __shared__ Job s_job;

    const uint32_t tid = threadIdx.x;
    if (tid < 64) {
        const uint32_t k = wave_job_of_unit(jl, blockIdx.x);
        if (tid == 0) s_job = job_at(jl, k);
    }
    __syncthreads();
    const HC_G DevTables *__restrict__ tb = (const HC_G DevTables *)s_job.tb;
    const HC_G uint32_t *__restrict__ in32 = (const HC_G uint32_t *)s_job.in;
    const uint64_t in_bytes = s_job.in_bytes, n = s_job.n;
    const uint64_t nb = num_blocks_dev(n, B);
    const HC_G uint64_t *__restrict__ off = (const HC_G uint64_t *)s_job.block_off;
    const HC_G uint32_t *__restrict__ sub_idx = (const HC_G uint32_t *)s_job.sub_idx;
    HC_G uint8_t *__restrict__ out = (HC_G uint8_t *)s_job.out;
    const uint32_t K = tb->lut_bits;
    const uint32_t max_len = tb->max_len;
    for (uint32_t k = tid; k < (1u << K); k += kDecThreads) s_lut[k] = tb->lut[k];
    for (uint32_t k = tid; k <= (uint32_t)kMaxLen; k += kDecThreads) {
        s_first[k] = tb->first[k];
        s_count[k] = tb->count[k];
        s_base[k] = tb->base[k];
    }
    s_sorted[tid] = tb->sorted[tid];
    __syncthreads();

    const uint64_t g = (uint64_t)(blockIdx.x - s_job.unit_begin) * kDecThreads + tid;
    const uint64_t i = g / cpb;
    const uint32_t c = (uint32_t)(g - i * cpb);
    if (i >= nb) return;
    const uint64_t blk_start = i * (uint64_t)B;
    const uint64_t left = n - blk_start;
    const uint32_t cnt = (uint32_t)(left < B ? left : B);
    const uint32_t s0 = c * S_eff;
    if (s0 >= cnt) return;
    const uint32_t s1 = (cnt - s0 < S_eff) ? cnt : s0 + S_eff;

    const uint64_t o = off[i], o1 = off[i + 1];
    if ((o & 3) || o + 4 > in_bytes || o1 > in_bytes || o1 < o + 4) {
        report(err, HC_ERR_CORRUPT);
        return;
    }
    if (c == 0 && ((i == 0 && o != 0) || (i + 1 == nb && o1 != in_bytes))) report(err, HC_ERR_CORRUPT);
    const uint32_t hdr = in32[o >> 2];
    if (o + 4 + 4 * (((uint64_t)hdr + 31) / 32) != o1) {
        report(err, HC_ERR_CORRUPT);
        return;
    }
    const HC_G uint32_t *payload = in32 + (o >> 2) + 1;
    const uint32_t nwords = (uint32_t)(((uint64_t)hdr + 31) >> 5);
    uint64_t p0 = 0, p1 = hdr;
    if (sub_idx) {
        p0 = sub_idx[i * cpb + c];
        if (s1 < cnt) p1 = sub_idx[i * cpb + c + 1];
    }
    if (p0 > p1 || p1 > hdr) {
        report(err, HC_ERR_CORRUPT);
        return;
    }

    BitReader br;
    br.seek(payload, nwords, p0);
    bool bad = false;
    HC_G uint8_t *dst = out + blk_start;
    uint32_t k = s0;
    for (; k + 16 <= s1 && !bad; k += 16) {
        uint32_t o4[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (uint32_t q = 0; q < 16; ++q) {
            const uint32_t sym = decode_one(br, payload, nwords, s_lut, K, max_len, s_first, s_count,
                                            s_base, s_sorted, bad);
            o4[q >> 2] |= sym << (8 * (q & 3));
        }
        *(HC_G v4u *)(dst + k) = v4u{o4[0], o4[1], o4[2], o4[3]};
    }
    for (; k < s1 && !bad; ++k)
        dst[k] = (uint8_t)decode_one(br, payload, nwords, s_lut, K, max_len, s_first, s_count, s_base,
                                     s_sorted, bad);
    if (bad || br.pos() != p1) {
        report(err, HC_ERR_CORRUPT);
        return;
    }
    if (s1 == cnt && (hdr & 31u)) {
        const uint32_t mask = (1u << (32 - (hdr & 31u))) - 1u;
        if (payload[nwords - 1] & mask) report(err, HC_ERR_CORRUPT);
    }
}

// ---------------------------------------------------------------- decode without the sub-block index
// One work-group per block; its lanes cut the block's payload bits into equal
// pieces and decode them in parallel without knowing where a code starts in
// a piece.  Section 2.1 recalls that a code stream cut at a fixed bit decodes
// wrongly from the cut, and that Huffman codes tend to fall back onto the
// true code boundaries soon after such a wrong start.  So each lane first
// decodes its piece from the piece's first bit: the codes that start before
// the piece's end, recording where the last of them ends (at or after the
// piece's end) and how many there were.  Then, round after round, a lane
// whose start differs from where its left neighbour's codes end decodes
// again from there.  Lane 0 starts on a true boundary, so after at most one
// round per lane every start is a true code boundary; usually one round
// settles all, since a re-decoded path meets the first one before the
// piece's end and the end no longer moves.  A scan of the counts places each
// piece's symbols, and each lane decodes its piece once more into the
// output.  The strict decoder's checks hold: every code valid, the codes end
// exactly at the header's bit count, their number is the block's symbol
// count, and the pad bits are zero.
constexpr uint32_t kSyncThreads = 256;
constexpr uint64_t kSyncMinPieceBits = 256;  // shorter pieces would spend most of their codes resynchronising
constexpr uint32_t kSyncStageWords = 16384;  // a block payload of up to 64 KiB is read from an LDS copy

// Codes that all fit the table (max_len <= lut_bits), positions below 2^31:
// one table read, a shift and a branch-free refill per code, 32-bit
// positions.  An invalid prefix reads as a 1-bit entry with kLutBadFlag, so
// every step advances; callers collect the flags.
struct TableBits {
    uint64_t buf;  // the next nb payload bits, most significant first
    uint32_t nb, wi, pos;

    template <typename Ptr>
    __device__ __forceinline__ void seek(Ptr src, uint32_t nwords, uint32_t p)
    {
        pos = p;
        wi = p >> 5;
        const uint32_t r = p & 31;
        buf = (((uint64_t)ld_word(src, nwords, wi) << 32) | ld_word(src, nwords, wi + 1)) << r;
        nb = 64 - r;
        wi += 2;
    }
    template <typename Ptr>
    __device__ __forceinline__ uint32_t next(Ptr src, uint32_t nwords, const uint16_t *lut, uint32_t K)
    {
        const uint32_t e = lut[(uint32_t)(buf >> (64 - K))];
        const uint32_t L = e & 0x7Fu;
        buf <<= L;
        nb -= L;
        pos += L;
        const bool need = nb < 32;  // nb >= 32 again after it: >= K bits for the next read
        const uint32_t w = need ? ld_word(src, nwords, wi) : 0u;
        buf |= (uint64_t)w << ((32 - nb) & 63);
        nb += need ? 32u : 0u;
        wi += need ? 1u : 0u;
        return e;
    }
};

// The pieces of one block, from its payload 'src' (global memory or its LDS
// copy); every lane of the group calls it (it holds barriers).
template <typename Ptr>
__device__ __forceinline__ void sync_block(Ptr src, uint32_t nwords, uint32_t hdr, uint32_t cnt,
                                           HC_G uint8_t *blk_out, uint32_t *err, const uint16_t *s_lut, uint32_t K,
                                           uint32_t max_len, const uint64_t *s_first, const uint32_t *s_count,
                                           const uint32_t *s_base, const uint32_t *s_sorted, uint64_t *s_end,
                                           uint32_t *s_scan)
{
    const uint32_t tid = threadIdx.x;
    const uint64_t bits = hdr;
    // pieces of L bits, at most one per lane: an odd number of 32-bit words,
    // so that the lanes' first reads of the LDS copy fall on distinct banks
    // (an even stride such as 64 words put all 64 lanes of a wave on one bank)
    uint64_t Lw = (bits + 32 * kSyncThreads - 1) / (32 * kSyncThreads);
    Lw = Lw < kSyncMinPieceBits / 32 ? kSyncMinPieceBits / 32 : Lw;
    Lw |= 1;
    const uint64_t L = 32 * Lw;
    const uint32_t np = (uint32_t)((bits + L - 1) / L);
    const bool mine = tid < np;
    const uint64_t lo = (uint64_t)tid * L;
    const uint64_t hi = lo + L < bits ? lo + L : bits;

    // the codes that start in [from, hi): their number and where they end;
    // every code read takes at least one bit, and an invalid prefix stops it
    // (the table loop reads it as a 1-bit code and flags it)
    // the codes that start in [from, hi): their number and where they end;
    // every code read takes at least one bit, and an invalid prefix stops it
    // (the table loop reads it as a 1-bit code and flags it)
    const bool table_only = max_len <= K && bits < (1ull << 31);  // the same in every lane
    auto run = [&](uint64_t from, uint32_t &c, bool &bad) -> uint64_t {
        if (table_only) {
            TableBits tbits;
            tbits.seek(src, nwords, (uint32_t)from);
            const uint32_t end = (uint32_t)hi;
            uint32_t n = 0, flags = 0;
            while (tbits.pos < end) {
                flags |= tbits.next(src, nwords, s_lut, K);
                ++n;
            }
            c = n;
            bad = (flags & kLutBadFlag) != 0;
            return tbits.pos;
        }
        BitReader br;
        br.seek(src, nwords, from);
        c = 0;
        bad = false;
        while (br.pos() < hi && !bad) {
            (void)decode_one(br, src, nwords, s_lut, K, max_len, s_first, s_count, s_base, s_sorted, bad);
            c += bad ? 0u : 1u;
        }
        return br.pos();
    };

    uint64_t start = lo;
    uint32_t c = 0;
    bool bad = false;
    if (mine) s_end[tid] = run(start, c, bad);
    __syncthreads();
    for (;;) {  // at most np + 1 rounds: lane j's start is final after j rounds
        const uint64_t t = (mine && tid > 0) ? s_end[tid - 1] : start;
        __syncthreads();  // every read of this round before any write
        bool moved = false;
        if (mine && tid > 0 && t != start) {
            start = t;
            s_end[tid] = run(start, c, bad);
            moved = true;
        }
        if (!__syncthreads_or(moved)) break;
    }

    uint32_t total = 0;
    const uint32_t first = group_exclusive_scan<uint32_t, kSyncThreads>(mine ? c : 0u, s_scan, &total);
    const bool any_bad = __syncthreads_or(mine && bad);
    const uint64_t last_end = np ? s_end[np - 1] : 0;
    if (any_bad || total != cnt || last_end != bits) {
        if (tid == 0) report(err, HC_ERR_CORRUPT);
        return;
    }
    if (tid == 0 && (hdr & 31u)) {
        const uint32_t mask = (1u << (32 - (hdr & 31u))) - 1u;
        if (src[nwords - 1] & mask) report(err, HC_ERR_CORRUPT);
    }
    if (!mine || c == 0) return;

    // the piece's symbols into blk_out[first, first + c): whole words where aligned
    BitReader br;
    TableBits tbits;
    if (table_only)
        tbits.seek(src, nwords, (uint32_t)start);
    else
        br.seek(src, nwords, start);
    HC_G uint8_t *dst = blk_out + first;
    bool unused = false;
    auto next = [&]() -> uint32_t {
        if (table_only) return tbits.next(src, nwords, s_lut, K) >> 8;
        return decode_one(br, src, nwords, s_lut, K, max_len, s_first, s_count, s_base, s_sorted, unused);
    };
    uint32_t k = 0;
    for (; k < c && ((uint64_t)(dst + k) & 3u); ++k) dst[k] = (uint8_t)next();
    for (; k + 4 <= c; k += 4) {
        uint32_t w = next();
        w |= next() << 8;
        w |= next() << 16;
        w |= next() << 24;
        *(HC_G uint32_t *)(dst + k) = w;
    }
    for (; k < c; ++k) dst[k] = (uint8_t)next();
}

// Work-group u decodes block u - unit_begin of the job that owns unit u (one
// unit per block: a batch of streams is one launch).  stage_words: the LDS
// words the launch gives the payload copy (a block whose payload is longer
// is read from global memory); shape_len: the longest code the launch was
// shaped for.
__global__ __launch_bounds__(kSyncThreads) void k_decode_sync(JobList jl, uint32_t B, uint32_t stage_words,
                                                               uint32_t shape_len, uint32_t *err)
{
    extern __shared__ uint32_t s_pay[];
    __shared__ uint16_t s_lut[1 << kLutBits];
    __shared__ uint64_t s_first[kMaxLen + 1];
    __shared__ uint32_t s_count[kMaxLen + 1];
    __shared__ uint32_t s_base[kMaxLen + 1];
    __shared__ uint32_t s_sorted[kNumSym];
    __shared__ uint64_t s_end[kSyncThreads];  // where lane j's codes end
    __shared__ uint32_t s_scan[kSyncThreads / 64];
    __shared__ Job s_job;

    const uint32_t tid = threadIdx.x;
    if (tid < 64) {
        const uint32_t k = wave_job_of_unit(jl, blockIdx.x);
        if (tid == 0) s_job = job_at(jl, k);
    }
    __syncthreads();
    const HC_G DevTables *__restrict__ tb = (const HC_G DevTables *)s_job.tb;
    const HC_G uint32_t *__restrict__ in32 = (const HC_G uint32_t *)s_job.in;
    const HC_G uint64_t *__restrict__ off = (const HC_G uint64_t *)s_job.block_off;
    HC_G uint8_t *__restrict__ out = (HC_G uint8_t *)s_job.out;
    const uint64_t in_bytes = s_job.in_bytes, n = s_job.n;
    const uint32_t K = tb->lut_bits;
    const uint32_t max_len = tb->max_len;
    if (max_len > shape_len) {  // the tables changed since the launch was shaped (the same in every lane)
        if (tid == 0) report(err, HC_ERR_TABLE_CHANGED);
        return;
    }
    for (uint32_t k = tid; k < (1u << K); k += kSyncThreads) s_lut[k] = tb->lut[k];
    for (uint32_t k = tid; k <= (uint32_t)kMaxLen; k += kSyncThreads) {
        s_first[k] = tb->first[k];
        s_count[k] = tb->count[k];
        s_base[k] = tb->base[k];
    }
    s_sorted[tid] = tb->sorted[tid];

    // the block and its checks (the same values in every lane: the group
    // leaves together or not at all)
    const uint64_t nb = num_blocks_dev(n, B);
    const uint64_t i = blockIdx.x - s_job.unit_begin;
    const uint64_t blk_start = i * (uint64_t)B;
    const uint32_t cnt = (uint32_t)(n - blk_start < B ? n - blk_start : B);
    const uint64_t o = off[i], o1 = off[i + 1];
    if ((o & 3) || o + 4 > in_bytes || o1 > in_bytes || o1 < o + 4) {
        if (tid == 0) report(err, HC_ERR_CORRUPT);
        return;
    }
    if (tid == 0 && ((i == 0 && o != 0) || (i + 1 == nb && o1 != in_bytes))) report(err, HC_ERR_CORRUPT);
    const uint32_t hdr = in32[o >> 2];
    if (o + 4 + 4 * (((uint64_t)hdr + 31) / 32) != o1) {
        if (tid == 0) report(err, HC_ERR_CORRUPT);
        return;
    }
    const HC_G uint32_t *payload = in32 + (o >> 2) + 1;
    const uint32_t nwords = (uint32_t)(((uint64_t)hdr + 31) >> 5);
    const bool staged = nwords <= stage_words;  // the same in every lane
    if (staged) {
        // 16 loads in flight per thread before their LDS stores: a copy
        // that waited for each load in turn took most of the kernel's time
        constexpr uint32_t kU = 16;
        for (uint32_t base = 0; base < nwords; base += kU * kSyncThreads) {
            uint32_t v[kU];
#pragma unroll
            for (uint32_t u = 0; u < kU; ++u) {
                const uint32_t w = base + u * kSyncThreads + tid;
                v[u] = w < nwords ? payload[w] : 0u;
            }
#pragma unroll
            for (uint32_t u = 0; u < kU; ++u) {
                const uint32_t w = base + u * kSyncThreads + tid;
                if (w < nwords) s_pay[w] = v[u];
            }
        }
    }
    __syncthreads();  // tables and the payload copy in LDS
    if (staged)
        sync_block((const uint32_t *)s_pay, nwords, hdr, cnt, out + blk_start, err, s_lut, K, max_len, s_first,
                   s_count, s_base, s_sorted, s_end, s_scan);
    else
        sync_block(payload, nwords, hdr, cnt, out + blk_start, err, s_lut, K, max_len, s_first, s_count, s_base,
                   s_sorted, s_end, s_scan);
}

// ---------------------------------------------------------------- decode, codes of <= 24 bits
// Same lane mapping and checks as k_decode; what differs is how a lane meets
// HBM.  Thousands of lanes each stream their own chunk, so a lane that read or
// wrote 16 bytes at a time would leave partly used 128-byte lines in L2 long
// enough to be evicted and fetched (or written) again.  Here every access of
// a lane is a whole line: compressed input arrives a 128-byte line at a time
// (8 consecutive 16-byte loads) into a private LDS ring, and decoded output is
// gathered in registers and stored a line at a time.
constexpr uint32_t kRingWords = 64;               // four 16-word halves: two lines
// Where a decode lane's output rounds that fall outside its chunk are stored
// (16 bytes per lane of a work-group; the contents are never read).
__device__ __attribute__((aligned(16))) uint8_t g_decode_sink[kDecThreads * 16];
constexpr uint32_t kRingStride = kRingWords + 1;  // odd stride: lanes spread over the banks

// Stream quad q (16 bytes), with q clamped to [0, q_last] (q_last at most the
// quad of the stream's last word): one load, no branch, so nothing waits for
// it before its data is used.  The stream is 16-byte aligned, so the quad of
// its last word lies in the same page and may be read whole; the words a
// clamped request stands in for only ever reach bit-buffer positions after a
// chunk's last code, which no decoded symbol depends on.
__device__ __forceinline__ v4u load_quad(const HC_G uint32_t *__restrict__ in32, int64_t q, int64_t q_last)
{
    q = q < 0 ? 0 : (q > q_last ? q_last : q);
    return *(const HC_G v4u *)(in32 + 4 * q);
}

// R symbols per round (8 or 16); refills of the bit buffer follow symbols
// SPR, 2*SPR, ... of a round and its last symbol (SPR * max_len <= 32);
// kLong: codes may be longer than the table.  kCopyOnly: every job of the
// launch has a complete 8-bit code, so only the copy form below runs and the
// ring is left out (its LDS would hold the copy to 2 groups per CU).
template <uint32_t R, uint32_t SPR, bool kLong, bool kCopyOnly = false>
__global__ __launch_bounds__(kDecThreads) void k_decode_ring(JobList jl, uint32_t B, uint32_t S_eff, uint32_t cpb,
                                                             uint32_t shape_len, uint32_t *err)
{
    constexpr uint32_t kRoundWords = R / 4;             // output words of a round
    constexpr uint32_t kLineRounds = 128 / R;           // rounds of one 128-byte output line
    extern __shared__ uint16_t s_lut[];  // 2^lut_bits entries (the launch sizes it for the largest)
    __shared__ uint32_t s_ring[kCopyOnly ? 1 : kDecThreads * kRingStride];
    __shared__ uint32_t s_first[kPackedMaxLen + 1];
    __shared__ uint32_t s_count[kPackedMaxLen + 1];
    __shared__ uint32_t s_base[kPackedMaxLen + 1];
    __shared__ uint32_t s_sorted[kNumSym];
    __shared__ Job s_job;

    const uint32_t tid = threadIdx.x;
    if (tid < 64) {
        const uint32_t k = wave_job_of_unit(jl, blockIdx.x);
        if (tid == 0) s_job = job_at(jl, k);
    }
    __syncthreads();
    const HC_G DevTables *__restrict__ tb = (const HC_G DevTables *)s_job.tb;
    const HC_G uint32_t *__restrict__ in32 = (const HC_G uint32_t *)s_job.in;
    const uint64_t in_bytes = s_job.in_bytes, n = s_job.n;
    const uint64_t nb = num_blocks_dev(n, B);
    const HC_G uint64_t *__restrict__ off = (const HC_G uint64_t *)s_job.block_off;
    const HC_G uint32_t *__restrict__ sub_idx = (const HC_G uint32_t *)s_job.sub_idx;
    HC_G uint8_t *__restrict__ out = (HC_G uint8_t *)s_job.out;
    const uint32_t K = tb->lut_bits;
    const uint32_t max_len = tb->max_len;
    const bool fixed8 = tb->fixed_len == 8;  // uniform over the group: one job per group
    // the tables must still be those the launch was shaped for (the same in every lane)
    if (max_len > shape_len || (kCopyOnly && !(fixed8 && tb->count[8] == (uint32_t)kNumSym))) {
        if (tid == 0) report(err, HC_ERR_TABLE_CHANGED);
        return;
    }
    if (!fixed8)
        for (uint32_t k = tid; k < (1u << K); k += kDecThreads) s_lut[k] = tb->lut[k];
    if (tid <= (uint32_t)kPackedMaxLen) {
        s_first[tid] = (uint32_t)tb->first[tid];
        s_count[tid] = tb->count[tid];
        s_base[tid] = tb->base[tid];
    }
    s_sorted[tid] = tb->sorted[tid];
    __syncthreads();  // the last barrier: lanes may leave early from here on

    // ---- the lane's chunk and its checks.  A lane without a chunk, or whose
    // chunk fails a check, stays until the complete-code copy below (which
    // every lane of a wave takes part in) and leaves after it.
    const uint64_t g = (uint64_t)(blockIdx.x - s_job.unit_begin) * kDecThreads + tid;
    const uint64_t i = g / cpb;
    const uint32_t c = (uint32_t)(g - i * cpb);
    bool ok = i < nb;
    uint64_t blk_start = 0, o = 0, o1 = 0, p0 = 0, p1 = 0;
    uint32_t cnt = 0, s0 = 0, s1 = 0, hdr = 0, nwords = 0;
    if (ok) {
        blk_start = i * (uint64_t)B;
        const uint64_t left = n - blk_start;
        cnt = (uint32_t)(left < B ? left : B);
        s0 = c * S_eff;
        ok = s0 < cnt;
    }
    if (ok) {
        s1 = (cnt - s0 < S_eff) ? cnt : s0 + S_eff;
        o = off[i];
        o1 = off[i + 1];
        if ((o & 3) || o + 4 > in_bytes || o1 > in_bytes || o1 < o + 4) {
            report(err, HC_ERR_CORRUPT);
            ok = false;
        }
    }
    if (ok) {
        if (c == 0 && ((i == 0 && o != 0) || (i + 1 == nb && o1 != in_bytes))) report(err, HC_ERR_CORRUPT);
        hdr = in32[o >> 2];
        if (o + 4 + 4 * (((uint64_t)hdr + 31) / 32) != o1) {
            report(err, HC_ERR_CORRUPT);
            ok = false;
        }
    }
    if (ok) {
        nwords = (uint32_t)(((uint64_t)hdr + 31) >> 5);
        p1 = hdr;
        if (sub_idx) {
            p0 = sub_idx[i * cpb + c];
            if (s1 < cnt) p1 = sub_idx[i * cpb + c + 1];
        } else if (fixed8) {  // chunks of a code whose lengths are all 8: at bit 8 s0 without an index
            p0 = 8ull * s0;
            if (s1 < cnt) p1 = 8ull * s1;
        }
        if (p0 > p1 || p1 > hdr) {
            report(err, HC_ERR_CORRUPT);
            ok = false;
        }
    }
    if (ok && fixed8 && (p0 != 8ull * s0 || p1 != 8ull * s1 || hdr != 8ull * cnt)) {
        // all codes are 8 bits: the index, the header and the pad must agree
        report(err, HC_ERR_CORRUPT);
        ok = false;
    }
    const uint64_t pw0 = (o >> 2) + 1;  // stream word of payload bit 0

    if (fixed8 && s_count[8] == kNumSym) {
        // All 256 bytes coded (a complete code: 2^8 codes of 8 bits): canonical
        // order is value order, every symbol is its own code, and a chunk
        // decodes as a copy of its payload words, each byte-swapped (the
        // first symbol is a word's top byte).  The wave copies its 64 chunks
        // together, 16 bytes per lane, so that each load and store instruction
        // moves a contiguous 1 KiB instead of 64 lanes touching 64 places;
        // every lane keeps four such pieces in flight.  A chunk starts on a
        // word (S is a multiple of 16) and its output on 16 bytes.
        if (ok && s1 == cnt && (hdr & 31u)) {
            const uint32_t mask = (1u << (32 - (hdr & 31u))) - 1u;
            if (in32[pw0 + nwords - 1] & mask) report(err, HC_ERR_CORRUPT);
        }
        const uint32_t lane = tid & 63u;
        const uint64_t src_w = pw0 + (s0 >> 2);                  // stream word of the chunk's first symbol
        const uint64_t dst_a = (uint64_t)(out + blk_start + s0);  // 16-byte aligned
        const uint32_t okns = ok ? s1 - s0 : 0u;                  // symbols to copy (0: none)
        {
            // The usual case: the wave's 64 chunks whole and in one block, so
            // its payload words and its output are each one contiguous range
            // (consecutive chunks of a block are consecutive in both).  Lane l
            // then copies words l + 64 m, every load and store instruction a
            // contiguous 256 bytes, with all of the lane's words (32 at
            // S = 128) in flight at once and no per-piece lane exchange.
            // (every lane of the wave is here: lane 0's values are read directly)
            const uint32_t i_lo = (uint32_t)i, i0 = (uint32_t)__builtin_amdgcn_readlane(i_lo, 0);
            if (__all(ok && okns == S_eff && i_lo == i0 && (uint32_t)(i >> 32) == 0u)) {
                const uint64_t s_w0 = read_lane_u64(src_w, 0);
                const uint64_t d_a0 = read_lane_u64(dst_a, 0);
                const HC_G uint32_t *src = in32 + s_w0 + lane;
                HC_G uint32_t *dst = (HC_G uint32_t *)d_a0 + lane;
                const uint32_t per_lane = S_eff / 4;  // words of the wave / 64
                constexpr uint32_t kU = 32;
                for (uint32_t m0 = 0; m0 < per_lane; m0 += kU) {
                    uint32_t v[kU];
#pragma unroll
                    for (uint32_t u = 0; u < kU; ++u)
                        if (m0 + u < per_lane) v[u] = src[64 * (m0 + u)];
#pragma unroll
                    for (uint32_t u = 0; u < kU; ++u)
                        if (m0 + u < per_lane) dst[64 * (m0 + u)] = __builtin_bswap32(v[u]);
                }
                return;
            }
        }
        const uint32_t pc = S_eff / 16;                           // 16-symbol pieces of a full chunk
        const uint32_t total = 64 * pc;                           // pieces of the wave's chunks
        for (uint32_t base = 0; base < total; base += 4 * 64) {
            uint32_t v[4][4];
            uint64_t d[4];
            uint32_t m[4];  // symbols of the piece to store: 16 (whole), 1..15 (a chunk's ragged end), 0
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u) {
                const uint32_t P = base + 64 * u + lane;
                const uint32_t j = (P < total ? P : 0u) / pc;  // the chunk (its lane in the wave)
                const uint32_t q = (P < total ? P : 0u) - j * pc;
                const uint32_t nsj = __shfl(okns, (int)j, 64);
                const uint64_t swj = ((uint64_t)__shfl((uint32_t)(src_w >> 32), (int)j, 64) << 32) |
                                     __shfl((uint32_t)src_w, (int)j, 64);
                d[u] = (((uint64_t)__shfl((uint32_t)(dst_a >> 32), (int)j, 64) << 32) |
                        __shfl((uint32_t)dst_a, (int)j, 64)) + 16ull * q;
                const uint32_t first = 16 * q;
                m[u] = (P < total && first < nsj) ? (nsj - first < 16 ? nsj - first : 16u) : 0u;
#pragma unroll
                for (uint32_t t = 0; t < 4; ++t)
                    v[u][t] = (4 * t < m[u]) ? in32[swj + 4 * q + t] : 0u;  // words holding the piece's symbols
            }
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u) {
                if (m[u] == 16) {
                    *(HC_G v4u *)d[u] = v4u{__builtin_bswap32(v[u][0]), __builtin_bswap32(v[u][1]),
                                            __builtin_bswap32(v[u][2]), __builtin_bswap32(v[u][3])};
                } else {
                    for (uint32_t k = 0; k < m[u]; ++k)
                        ((HC_G uint8_t *)d[u])[k] = (uint8_t)(v[u][k >> 2] >> (24 - 8 * (k & 3)));
                }
            }
        }
        return;
    }
    if (kCopyOnly) return;  // not reached: the launch holds complete 8-bit codes only (checked above)
    if (!ok) return;

    // ---- input ring.  Stream words are counted from the 128-byte line that
    // holds the stream's first word (virtual word = stream word + mis), and
    // from the line of the chunk's first bit on in 32 bits ('local' words
    // below; local line l = local words [32l, 32l + 32)).  The ring holds the
    // local words of halves [nxt / 16, vend) (16 words each, word w at slot
    // w mod 64): up to four halves, two lines.
    //
    // A wait for a global load stalls the whole wave, and lanes need their
    // lines at different times.  So lines are requested only at sync points,
    // every fourth round (rounds 2 and 6 of an output line, away from the line
    // stores, which a wait would also cover), by all lanes together: each lane
    // requests the line after its ring's end into registers f, and at a
    // later sync point (four rounds on or more, when the load has landed)
    // moves it into the ring once two halves are free and requests the next.
    // The line waits in registers meanwhile: requesting it again would find
    // it evicted from L2 as often as not, with thousands of lanes streaming.  Four rounds
    // consume at most 32 words (4 * R * max_len <= 1024 bits), and after a
    // sync point the ring holds at least three halves from the current word
    // on, so a round never reads a word the ring does not hold.
    const uint64_t in_words = in_bytes >> 2;
    const uint32_t mis = (uint32_t)(((uint64_t)in32 >> 2) & 31u);  // a multiple of 4
    const uint64_t u0 = pw0 + (p0 >> 5) + mis;                     // virtual word of the chunk's first bit
    const uint64_t ubase = u0 & ~(uint64_t)31;                     // virtual word of local word 0
    const int64_t qbase = (int64_t)(ubase >> 2) - (int64_t)(mis >> 2);  // stream quad of local quad 0
    uint32_t *ring = s_ring + tid * kRingStride;
    // Requests stop at the quad of the chunk's last payload word: a line past
    // it would only fill bit-buffer positions after the chunk's last code, and
    // is the next chunk's, read by its lane long before, so it would come from
    // HBM a second time.  Clamped requests hit the lane's own recent line.
    const uint64_t w_last = pw0 + (p1 ? (p1 - 1) >> 5 : 0);
    const int64_t q_last = (int64_t)((w_last < in_words ? w_last : in_words - 1) >> 2);
    auto load_line = [&](uint32_t l, v4u f[8]) {
#pragma unroll
        for (uint32_t j = 0; j < 8; ++j) f[j] = load_quad(in32, qbase + 8 * (int64_t)l + j, q_last);
    };
    auto put_line = [&](uint32_t l, const v4u f[8]) {  // local line l into its two ring halves
#pragma unroll
        for (uint32_t j = 0; j < 8; ++j) {
            const uint32_t w = 32 * l + 4 * j;
            ring[(w + 0) & 63u] = f[j].x;
            ring[(w + 1) & 63u] = f[j].y;
            ring[(w + 2) & 63u] = f[j].z;
            ring[(w + 3) & 63u] = f[j].w;
        }
    };
    uint32_t nxt = (uint32_t)(u0 - ubase);  // next local word to enter the bit buffer (< 32)
    uint32_t vend = 4;                      // halves [0, 4) are in the ring after the set-up
    v4u f[8];
    {
        // Nothing may be pending when the loops start: a load still pending
        // there would make the compiler's waits for f in the loops count only
        // the loads behind it, and so also wait for the line stores issued
        // since the previous sync round.  So line 2 is requested first and
        // waited for (the empty asm) with lines 0 and 1.
        v4u a[8], b[8];
        load_line(2, f);
        load_line(0, a);
        load_line(1, b);
        put_line(0, a);
        put_line(1, b);
#pragma unroll
        for (uint32_t j = 0; j < 8; ++j) asm volatile("" ::"v"(f[j].x), "v"(f[j].y), "v"(f[j].z), "v"(f[j].w));
    }
    auto sync_lines = [&]() {
        if (vend - (nxt >> 4) <= 2) {  // two halves free: f (line vend / 2) moves in, the next line is requested
            put_line(vend >> 1, f);
            vend += 2;
            load_line(vend >> 1, f);
        }
    };

    // ---- output: a line of 128 bytes in registers, stored whole.  Round v
    // (counted from the line holding the chunk's first byte) fills words
    // [kRoundWords * (v mod kLineRounds), +kRoundWords) of line v / kLineRounds;
    // the rounds before the chunk's first byte and after its last full round
    // do not exist and are skipped.
    HC_G uint8_t *const dst = out + blk_start + s0;
    const uint32_t nsym = s1 - s0;
    const uint32_t ph = (uint32_t)((uint64_t)dst & 127u);  // a multiple of 16
    const uint32_t v_first = ph / R;                       // round of the chunk's first byte
    const uint32_t v_end = v_first + nsym / R;             // after the last full round
    HC_G uint8_t *const line0 = dst - ph;                  // the line holding the first byte
    //
    // A store's data registers may not be written again before the store has
    // completed, so the rounds of the next line must not write the registers
    // of the line being stored: the line is copied into st and stored from
    // there, and st is kept allocated until the next store (the empty asm),
    // one line of decoding later, by when the store has long completed.
    //
    // Every line issues all its stores: a round the lane does not own goes
    // to a sink instead of being skipped.  A path through the loop without
    // stores would make the compiler count, at the next wait for the line in
    // f, only the loads behind f, and so wait for these stores as well.
    uint32_t ow[32], st[32];
#pragma unroll
    for (uint32_t i = 0; i < 32; ++i) st[i] = 0;
    HC_G uint8_t *const sink = (HC_G uint8_t *)g_decode_sink + 16 * tid;
    auto store_line = [&](uint32_t lb) {  // the rounds [lb, lb + kLineRounds) that exist
#pragma unroll
        for (uint32_t i = 0; i < 32; i += 4) asm volatile("" ::"v"(st[i]), "v"(st[i + 1]), "v"(st[i + 2]), "v"(st[i + 3]));
#pragma unroll
        for (uint32_t i = 0; i < 32; ++i) st[i] = ow[i];
#pragma unroll
        for (uint32_t r = 0; r < kLineRounds; ++r) {
            const uint32_t v = lb + r;
            HC_G uint8_t *p = (v >= v_first && v < v_end) ? line0 + (uint64_t)R * v : sink;
            if (R == 16)
                *(HC_G v4u *)p = v4u{st[4 * r], st[4 * r + 1], st[4 * r + 2], st[4 * r + 3]};
            else
                *(HC_G v2u *)p = v2u{st[2 * r], st[2 * r + 1]};
        }
    };
    uint32_t k = 0;  // symbols of the full rounds

    if (fixed8) {
        // Every code is 8 bits: symbol q of a round is byte 3 - (q & 3) of
        // word nxt + q / 4 (a chunk starts on a word: S is a multiple of 16),
        // so a round is four ring words and sixteen table lookups.
        const uint32_t ncode = s_count[8];
        uint32_t bad8 = 0;
        auto code_at = [&](uint32_t q) -> uint32_t {
            const uint32_t cd = (ring[(nxt + (q >> 2)) & 63u] >> (24 - 8 * (q & 3))) & 255u;
            bad8 |= (uint32_t)(cd >= ncode);
            return cd;
        };
        for (uint32_t lb = v_first - v_first % kLineRounds; lb < v_end; lb += kLineRounds) {
#pragma unroll
            for (uint32_t r = 0; r < kLineRounds; ++r) {
                if (r % 8 == 2) sync_lines();  // 8 rounds take 32 words: one sync per line of output
                const uint32_t v = lb + r;
                if (v >= v_first && v < v_end) {
#pragma unroll
                    for (uint32_t q = 0; q < kRoundWords; ++q)
                        ow[kRoundWords * r + q] = s_sorted[code_at(4 * q)] | (s_sorted[code_at(4 * q + 1)] << 8) |
                                                  (s_sorted[code_at(4 * q + 2)] << 16) |
                                                  (s_sorted[code_at(4 * q + 3)] << 24);
                    nxt += R / 4;
                }
            }
            store_line(lb);
        }
        k = nsym - nsym % R;
        if (k < nsym) {  // fewer than R symbols: at most R/4 words from nxt
            sync_lines();
            for (uint32_t q = 0; q < nsym - k; ++q) dst[k + q] = (uint8_t)s_sorted[code_at(q)];
        }
        if (s1 == cnt && (hdr & 31u)) {
            const uint32_t mask = (1u << (32 - (hdr & 31u))) - 1u;
            bad8 |= (in32[pw0 + nwords - 1] & mask) ? 1u : 0u;
        }
        if (bad8) report(err, HC_ERR_CORRUPT);
        return;
    }

    // ---- bit buffer: the next nbits payload bits, most significant first;
    // 'pre' is the ring word at nxt, read ahead of its refill.
    const uint32_t r0 = (uint32_t)(p0 & 31);
    uint64_t buf = (((uint64_t)ring[nxt & 63u] << 32) | ring[(nxt + 1) & 63u]) << r0;
    uint32_t nbits = 64 - r0;
    nxt += 2;
    uint32_t pre = ring[nxt & 63u];
    uint32_t bad = 0;  // kLutBadFlag: an invalid prefix was met

    // One symbol from the buffer (which holds >= max_len bits here), as its
    // table entry (symbol << 8) | length.  Invalid prefixes carry kLutBadFlag
    // and a length of 1, so codes of at most lut_bits bits need no test;
    // longer codes (kLong) take the canonical-range search on the buffered
    // bits.  The lengths are summed as whole entries (esum): the symbols sit
    // above bit 8 and the at most SPR lengths summed between refills total
    // <= 32, so the low byte of the sum is their total.
    const uint32_t lut_shift = 32 - K;
    uint32_t esum = 0;
    auto decode_entry = [&]() -> uint32_t {
        uint32_t e = s_lut[(uint32_t)(buf >> 32) >> lut_shift];
        if (kLong && (e & 255u) == 0) {
            uint32_t L = 0, sym = 0;
            for (uint32_t l = K + 1; l <= max_len; ++l) {
                const uint32_t cv = (uint32_t)(buf >> (64 - l));
                const uint32_t d = cv - s_first[l];
                if (d < s_count[l]) {
                    L = l;
                    sym = s_sorted[s_base[l] + d];
                    break;
                }
            }
            e = L ? (sym << 8) | L : (kLutBadFlag | 1u);
        }
        bad |= e;
        buf <<= (e & 63u);
        esum += e;
        return e;
    };
    // Tops the buffer up to >= 32 bits with the word read ahead, without a
    // branch; the ring word after it is read for the next refill.
    auto refill = [&]() {
        nbits -= esum & 255u;
        esum = 0;
        const bool need = nbits < 32;
        const uint32_t w = need ? pre : 0u;
        buf |= (uint64_t)w << ((32 - nbits) & 63u);
        nbits += need ? 32u : 0u;
        nxt += need ? 1u : 0u;
        pre = ring[nxt & 63u];
    };

    for (uint32_t lb = v_first - v_first % kLineRounds; lb < v_end; lb += kLineRounds) {
#pragma unroll
        for (uint32_t r = 0; r < kLineRounds; ++r) {
            if (r % 4 == 2) sync_lines();
            const uint32_t v = lb + r;
            if (v >= v_first && v < v_end) {
                uint32_t o4[kRoundWords];
#pragma unroll
                for (uint32_t q = 0; q < kRoundWords; ++q) o4[q] = 0;
#pragma unroll
                for (uint32_t q = 0; q < R; ++q) {
                    // the entry's byte 1 (the symbol) into byte q & 3 of the word, the other bytes kept
                    constexpr uint32_t kSel[4] = {0x03020105u, 0x03020500u, 0x03050100u, 0x05020100u};
                    o4[q >> 2] = __builtin_amdgcn_perm(decode_entry(), o4[q >> 2], kSel[q & 3]);
                    if ((q + 1) % SPR == 0 || q + 1 == R) refill();
                }
#pragma unroll
                for (uint32_t q = 0; q < kRoundWords; ++q) ow[kRoundWords * r + q] = o4[q];
            }
        }
        store_line(lb);
    }
    k = nsym - nsym % R;
    if (k < nsym) {  // the ragged last round: one symbol between refills
        sync_lines();
        for (uint32_t q = 0; q < nsym - k; ++q) {
            dst[k + q] = (uint8_t)(decode_entry() >> 8);
            refill();
        }
    }
    const uint64_t pos = 32 * (ubase + nxt - mis - pw0) - nbits;
    if ((bad & kLutBadFlag) || pos != p1) {
        report(err, HC_ERR_CORRUPT);
        return;
    }
    if (s1 == cnt && (hdr & 31u)) {
        const uint32_t mask = (1u << (32 - (hdr & 31u))) - 1u;
        if (in32[pw0 + nwords - 1] & mask) report(err, HC_ERR_CORRUPT);
    }
}

// ---------------------------------------------------------------- decode, wave-staged chunks
// Same lane mapping, checks and table decode as k_decode_ring, for chunks of
// at most kStageMaxS symbols (the sub-block index with S <= 128); what
// differs is how a wave meets HBM.  The 64 chunks of a wave are consecutive
// in the stream (blocks are back to back and a block's chunks in order), so
// the wave copies the stream words they span into an LDS area of its own
// with coalesced 16-byte loads (each load instruction moves a contiguous
// 1 KiB), and then every lane decodes its chunk from there into 32 registers
// (one 128-byte line) stored once at the end.  No per-lane ring, no line in
// flight in registers and no rounds of the wave waiting for each other's
// lines: the state of a lane is its bit buffer and its output line, so more
// waves fit a CU (the per-symbol chain of table reads is latency-bound, and
// waves are what hides it).  If the words of the wave's chunks do not fit
// the area at once (long codes, or a corrupt index), the wave takes them in
// passes, each pass the pending lanes whose words fit after the lowest one.
constexpr uint32_t kStageMaxS = 128;     // symbols of a chunk: one 128-byte output line
constexpr uint32_t kStageSlackWords = 128;  // after the last wave's area: reads past a corrupt chunk's end stay in LDS
// Words of each wave's area: the 64 chunks at 8 bits per symbol, and at least
// the longest chunk the checks let through (kStageMaxS codes of 24 bits) with
// the bit buffer's read-ahead.  Static: the areas are fixed-size arrays.
constexpr uint32_t kStageWords = 64 * kStageMaxS / 4 + 16;
static_assert(kStageWords >= 32 * 36, "half a wave's output lines fit the area");
static_assert(kStageWords % 4 == 0 && kStageWords >= (kStageMaxS * kPackedMaxLen) / 32 + 16, "area too small");

// The minimum (maximum) of a 64-bit value over all 64 lanes, the same in
// every lane.  Data-parallel moves (DPP) instead of lane exchanges through
// the LDS unit: an inclusive scan within each row of 16 lanes (shifts by 1,
// 2, 4, 8), then row 0's result into row 1 and row 2's into row 3 (the
// broadcast of lane 15), then rows 0-1 into rows 2-3 (the broadcast of lane
// 31); lane 63 ends with the wave's result, read out as a scalar.  Every step
// is a VALU move, where each step of a lane exchange waited on an LDS round
// trip.  All 64 lanes must be active.
template <bool kMin>
__device__ __forceinline__ uint64_t wave_reduce_u64(uint64_t v)
{
    auto step = [&](auto ctrl, auto rows) {
        constexpr int kCtrl = decltype(ctrl)::value, kRows = decltype(rows)::value;
        // lanes without a source in range keep their own value
        const uint32_t lo = __builtin_amdgcn_update_dpp((uint32_t)v, (uint32_t)v, kCtrl, kRows, 0xF, false);
        const uint32_t hi =
            __builtin_amdgcn_update_dpp((uint32_t)(v >> 32), (uint32_t)(v >> 32), kCtrl, kRows, 0xF, false);
        const uint64_t o = ((uint64_t)hi << 32) | lo;
        v = kMin ? (o < v ? o : v) : (o > v ? o : v);
    };
    using std::integral_constant;
    step(integral_constant<int, 0x111>(), integral_constant<int, 0xF>());  // row_shr:1
    step(integral_constant<int, 0x112>(), integral_constant<int, 0xF>());  // row_shr:2
    step(integral_constant<int, 0x114>(), integral_constant<int, 0xF>());  // row_shr:4
    step(integral_constant<int, 0x118>(), integral_constant<int, 0xF>());  // row_shr:8
    step(integral_constant<int, 0x142>(), integral_constant<int, 0xA>());  // row_bcast:15 into rows 1, 3
    step(integral_constant<int, 0x143>(), integral_constant<int, 0xC>());  // row_bcast:31 into rows 2, 3
    return read_lane_u64(v, 63);
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) { return wave_reduce_u64<true>(v); }
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) { return wave_reduce_u64<false>(v); }

// LDS written by some lanes of a wave, then read by others: the writes are
// complete before any lane reads.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The bit reader of one chunk in its wave's area: 'buf' holds the 64 area
// bits from the reader's position on (at least 33 of them the chunk's: two
// words shifted by the bit offset); the table entries decoded since the last refill are
// summed in esum, whose low byte is then their total length (refills come
// after at most SPR codes, SPR * max_len <= 32).  So the next window starts
// at most one word after this one: x0, x1 are this window's two area words
// and x2 the one after, read at the last refill, and a refill takes its
// words from them and reads only the next word ahead, so that no refill
// waits on LDS inside the chain of table reads.  kAhead false: each refill
// reads its two words (the two-chain kernels, whose registers the three
// words would overflow).
template <bool kAhead>
struct StageBits {
    uint64_t buf;
    uint32_t esum;
    uint32_t sh;         // the window's first bit inside x0 (0..31)
    const uint32_t *wp;  // the area word x0 is
    uint32_t x0, x1, x2;

    // p: the chunk's first bit, counted from the area's first word
    __device__ __forceinline__ void start(const uint32_t *area, uint32_t p, bool read)
    {
        wp = area + (p >> 5);
        sh = p & 31u;
        esum = 0;
        if (read) window();
    }
    __device__ __forceinline__ void window()
    {
        x0 = wp[0];
        x1 = wp[1];
        if (kAhead) x2 = wp[2];
        buf = (((uint64_t)x0 << 32) | x1) << sh;
    }
    // The word pointer and the bit offset are kept apart, so that a refill
    // needs no address arithmetic beyond one add: the read-ahead word is
    // wp[2] (an immediate offset) and the window shift is sh itself.
    __device__ __forceinline__ void refill()
    {
        sh += esum & 255u;
        esum = 0;
        const uint32_t step = sh >> 5;  // whole words passed: at most one unless the chunk is corrupt
        sh &= 31u;
        wp += step;
        if (!kAhead) {
            window();
            return;
        }
        const bool adv = step != 0;
        x0 = adv ? x1 : x0;
        x1 = adv ? x2 : x1;
        buf = (((uint64_t)x0 << 32) | x1) << sh;
        x2 = wp[2];
    }
    // the reader's bit position, counted from the area's first word
    __device__ __forceinline__ uint32_t position(const uint32_t *area) const { return 32u * (uint32_t)(wp - area) + sh; }
};

// One code from the reader: its symbol is returned (in byte 1 with kLong,
// else byte 0) and its length taken from the bit buffer.  Where every code fits the table (!kLong) it is kept
// as two byte tables, lengths and symbols, so that the chain from one code to
// the next (length read, shift of the buffer, next index) uses the index
// itself as the read address, and the symbol read is off that chain.  kLong:
// the table holds (symbol << 8) | length (length 0: a longer code), and codes
// longer than the table take the canonical-range search on the buffered bits
// (which hold >= max_len bits whenever a code starts); these launches keep
// the one table, whose registers fit them.  An invalid prefix reads as a
// 1-bit code flagged kLutBadFlag (or-ed into bad).
template <bool kLong, bool kAhead>
__device__ __forceinline__ uint32_t stage_entry(StageBits<kAhead> &b, const uint16_t *lut16, const uint8_t *lut_len,
                                                const uint8_t *lut_sym, uint32_t lut_shift, uint32_t K,
                                                uint32_t max_len, const uint32_t *s_first, const uint32_t *s_count,
                                                const uint32_t *s_base, const uint32_t *s_sorted, uint32_t &bad)
{
    const uint32_t i = (uint32_t)(b.buf >> 32) >> lut_shift;
    // kLong: the entry, symbol in byte 1; otherwise the length, and the symbol in byte 0
    uint32_t e, ret;
    if (kLong) {
        e = lut16[i];
        if ((e & 255u) == 0) {
            e = kLutBadFlag | 1u;
            for (uint32_t l = K + 1; l <= max_len; ++l) {
                const uint32_t cv = (uint32_t)(b.buf >> (64 - l));
                const uint32_t d = cv - s_first[l];
                if (d < s_count[l]) {
                    e = (s_sorted[s_base[l] + d] << 8) | l;
                    break;
                }
            }
        }
        ret = e;
    } else {
        e = lut_len[i];
        ret = lut_sym[i];
    }
    bad |= e;
    b.buf <<= (e & 63u);
    b.esum += e;
    return ret;
}

// The symbol (byte kB of s) into byte q & 3 of a word, the other bytes kept.
template <uint32_t kB>
__device__ __forceinline__ uint32_t put_sym(uint32_t s, uint32_t word, uint32_t q)
{
    constexpr uint32_t x = 4 + kB;  // byte kB of the first operand
    constexpr uint32_t kSel[4] = {0x03020100u & ~0xFFu | x, 0x03020100u & ~0xFF00u | (x << 8),
                                  0x03020100u & ~0xFF0000u | (x << 16), 0x03020100u & ~0xFF000000u | (x << 24)};
    return __builtin_amdgcn_perm(s, word, kSel[q & 3]);
}

// R symbols per round (16, or 8 for codes of 17..24 bits); refills follow
// symbols SPR, 2*SPR, ... of a round and its last symbol; kLong: codes may be
// longer than the table; kLutB: table entries of the launch (2^kLutB >=
// 2^lut_bits of every job).  kChains: consecutive chunks per lane (2 for
// chunks of <= 64 symbols: two independent decode chains interleaved, so
// each lane has two table reads in flight; 1 for chunks of 65..128).  A
// group always covers 256 chunks (256 / kChains lanes).  All LDS is static
// (about 8 KiB of area per wave).
template <uint32_t R, uint32_t SPR, bool kLong, uint32_t kLutB, uint32_t kChains>
__global__ __launch_bounds__(kDecThreads / kChains) __attribute__((amdgpu_waves_per_eu(kLutB <= 10 ? 4 : 3))) void k_decode_stage(
    JobList jl, uint32_t B, uint32_t S_eff, uint32_t cpb, uint32_t shape_len, uint32_t *err)
{
    constexpr uint32_t kThreads = kDecThreads / kChains;
    constexpr uint32_t kWaves = kThreads / 64;
    constexpr uint32_t kChainSyms = kStageMaxS / kChains;  // the longest chunk of the launch
    constexpr uint32_t kChainWords = kChainSyms / 4;       // its output words
    constexpr uint32_t kRoundWords = R / 4;
    constexpr uint32_t kChainRounds = kChainSyms / R;
    static_assert(kChainSyms % 16 == 0 && kChainSyms % R == 0, "whole 16-byte pieces per chunk");
    constexpr uint32_t kLutN = 1u << kLutB;
    __shared__ __attribute__((aligned(16))) uint16_t s_lut16[kLong ? kLutN : 8];    // kLong: the table as it is
    __shared__ __attribute__((aligned(16))) uint8_t s_lut_len[kLong ? 16 : kLutN];  // otherwise its length bytes
    __shared__ __attribute__((aligned(16))) uint8_t s_lut_sym[kLong ? 16 : kLutN];  // and symbol bytes
    __shared__ __attribute__((aligned(16))) uint32_t s_area[kWaves * kStageWords + kStageSlackWords];
    __shared__ uint32_t s_first[kPackedMaxLen + 1];
    __shared__ uint32_t s_count[kPackedMaxLen + 1];
    __shared__ uint32_t s_base[kPackedMaxLen + 1];
    __shared__ uint32_t s_sorted[kNumSym];
    __shared__ Job s_job;

    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    if (tid < 64) {
        const uint32_t k = wave_job_of_unit(jl, blockIdx.x);
        if (tid == 0) s_job = job_at(jl, k);
    }
    __syncthreads();
    const HC_G DevTables *__restrict__ tb = (const HC_G DevTables *)s_job.tb;
    const HC_G uint32_t *__restrict__ in32 = (const HC_G uint32_t *)s_job.in;
    const uint64_t in_bytes = s_job.in_bytes, n = s_job.n;
    const uint64_t nb = num_blocks_dev(n, B);
    const HC_G uint64_t *__restrict__ off = (const HC_G uint64_t *)s_job.block_off;
    const HC_G uint32_t *__restrict__ sub_idx = (const HC_G uint32_t *)s_job.sub_idx;
    HC_G uint8_t *__restrict__ out = (HC_G uint8_t *)s_job.out;
    const uint32_t K = tb->lut_bits;
    const uint32_t max_len = tb->max_len;
    if (max_len > shape_len) {  // the tables changed since the launch was shaped (the same in every lane)
        if (tid == 0) report(err, HC_ERR_TABLE_CHANGED);
        return;
    }
    {
        // the table, 8 entries (16 bytes) per load; without kLong split into
        // its length bytes (byte 0 of each entry) and symbol bytes (byte 1)
        const uint32_t nq = (1u << K) >= 8 ? (1u << K) / 8 : 1u;
        for (uint32_t k = tid; k < nq; k += kThreads) {
            const v4u v = ((const HC_G v4u *)tb->lut)[k];
            if (kLong) {
                ((v4u *)s_lut16)[k] = v;
            } else {
                *(v2u *)(s_lut_len + 8 * k) =
                    v2u{__builtin_amdgcn_perm(v.y, v.x, 0x06040200u), __builtin_amdgcn_perm(v.w, v.z, 0x06040200u)};
                *(v2u *)(s_lut_sym + 8 * k) =
                    v2u{__builtin_amdgcn_perm(v.y, v.x, 0x07050301u), __builtin_amdgcn_perm(v.w, v.z, 0x07050301u)};
            }
        }
    }
    if (tid <= (uint32_t)kPackedMaxLen) {
        s_first[tid] = (uint32_t)tb->first[tid];
        s_count[tid] = tb->count[tid];
        s_base[tid] = tb->base[tid];
    }
    for (uint32_t k = tid; k < (uint32_t)kNumSym; k += kThreads) s_sorted[k] = tb->sorted[k];
    __syncthreads();  // the last barrier of the group: waves go their own way from here

    // ---- the lane's chunks and their checks (as k_decode_ring, per chunk)
    const bool small_job = nb * cpb < (1ull << 32);  // chunk numbers fit 32 bits (the same in every lane)
    bool ok[kChains];
    uint64_t blk_start[kChains], pw0[kChains], fw[kChains], lw[kChains], p0[kChains], p1[kChains];
    uint32_t cnt[kChains], s0[kChains], s1[kChains], hdr[kChains], nwords[kChains];
#pragma unroll
    for (uint32_t h = 0; h < kChains; ++h) {
        const uint64_t g = ((uint64_t)(blockIdx.x - s_job.unit_begin) * kThreads + tid) * kChains + h;
        const uint64_t i = small_job ? (uint64_t)((uint32_t)g / cpb) : g / cpb;
        const uint32_t c = (uint32_t)(g - i * cpb);
        bool k_ok = i < nb;
        uint64_t o = 0, o1 = 0;
        blk_start[h] = 0; p0[h] = 0; p1[h] = 0;
        cnt[h] = 0; s0[h] = 0; s1[h] = 0; hdr[h] = 0; nwords[h] = 0;
        if (k_ok) {
            blk_start[h] = i * (uint64_t)B;
            const uint64_t left = n - blk_start[h];
            cnt[h] = (uint32_t)(left < B ? left : B);
            s0[h] = c * S_eff;
            k_ok = s0[h] < cnt[h];
        }
        if (k_ok) {
            s1[h] = (cnt[h] - s0[h] < S_eff) ? cnt[h] : s0[h] + S_eff;
            o = off[i];
            o1 = off[i + 1];
            if ((o & 3) || o + 4 > in_bytes || o1 > in_bytes || o1 < o + 4) {
                report(err, HC_ERR_CORRUPT);
                k_ok = false;
            }
        }
        if (k_ok) {
            if (c == 0 && ((i == 0 && o != 0) || (i + 1 == nb && o1 != in_bytes))) report(err, HC_ERR_CORRUPT);
            hdr[h] = in32[o >> 2];
            if (o + 4 + 4 * (((uint64_t)hdr[h] + 31) / 32) != o1) {
                report(err, HC_ERR_CORRUPT);
                k_ok = false;
            }
        }
        if (k_ok) {
            nwords[h] = (uint32_t)(((uint64_t)hdr[h] + 31) >> 5);
            p1[h] = hdr[h];
            p0[h] = sub_idx[i * cpb + c];
            if (s1[h] < cnt[h]) p1[h] = sub_idx[i * cpb + c + 1];
            // every code has 1 .. max_len bits
            const uint64_t ns = s1[h] - s0[h];
            if (p0[h] > p1[h] || p1[h] > hdr[h] || p1[h] - p0[h] < ns || p1[h] - p0[h] > ns * max_len) {
                report(err, HC_ERR_CORRUPT);
                k_ok = false;
            }
        }
        ok[h] = k_ok;
        pw0[h] = (o >> 2) + 1;                  // stream word of payload bit 0
        fw[h] = pw0[h] + (p0[h] >> 5);          // stream word of the chunk's first bit
        lw[h] = pw0[h] + ((p1[h] - 1) >> 5);    // and of its last bit
    }
    // the stream words the lane's chunks span
    uint64_t lo = ~0ull, hi = 0;
    bool pending = false;
#pragma unroll
    for (uint32_t h = 0; h < kChains; ++h) {
        if (ok[h]) {
            lo = fw[h] < lo ? fw[h] : lo;
            hi = lw[h] > hi ? lw[h] : hi;
            pending = true;
        }
    }
    const uint64_t in_words = in_bytes >> 2;
    const int64_t q_last = (int64_t)((in_words ? in_words - 1 : 0) >> 2);  // the stream's last quad
    uint32_t *const area = s_area + wave * kStageWords;
    constexpr uint32_t area_quads = kStageWords / 4;
    const uint32_t lut_shift = 32 - K;
    uint32_t bad = 0;  // kLutBadFlag: an invalid prefix was met

    while (__any(pending)) {
        // the pass: pending lanes whose words (and the three the bit buffer
        // reads ahead) fit the area from the lowest pending quad on
        const uint64_t bq = wave_min_u64(pending ? (lo >> 2) : ~0ull);
        const bool take = pending && ((hi + 3) >> 2) < bq + area_quads;
        const uint64_t eq = wave_max_u64(take ? ((hi + 3) >> 2) + 1 : 0ull);
        if (!__any(take)) {
            // not reached with a valid stream (a lane's chunks span far less
            // than an area); a corrupt one may, and no wave may loop forever
            if (pending && (lo >> 2) == bq) {
                report(err, HC_ERR_CORRUPT);
                pending = false;
            }
            continue;
        }
        // <= area_quads by the choice of 'take'; clamped all the same, so that
        // the copy below never writes past the wave's area
        const uint32_t nq = (uint32_t)(eq - bq < area_quads ? eq - bq : area_quads);
        {
            constexpr uint32_t kU = 8;  // loads in flight per lane: 8 KiB per wave
            for (uint32_t q0 = 0; q0 < nq; q0 += 64 * kU) {
                v4u v[kU];
#pragma unroll
                for (uint32_t u = 0; u < kU; ++u) {
                    const uint32_t q = q0 + 64 * u + lane;
                    v[u] = q < nq ? load_quad(in32, (int64_t)(bq + q), q_last) : v4u{0u, 0u, 0u, 0u};
                }
#pragma unroll
                for (uint32_t u = 0; u < kU; ++u) {
                    const uint32_t q = q0 + 64 * u + lane;
                    if (q < nq) *(v4u *)(area + 4 * q) = v[u];
                }
            }
        }
        wave_lds_sync();
        // every chunk of the wave whole and taken in this pass: the wave's
        // output is one contiguous range (a lane's chunks are consecutive, and
        // so are the lanes'), stored through the area afterwards
        bool whole = take;
#pragma unroll
        for (uint32_t h = 0; h < kChains; ++h) whole = whole && ok[h] && s1[h] - s0[h] == S_eff;
        const bool coalesce = __all(whole) && S_eff * kChains == kStageMaxS;
        if (take) {
            StageBits<kChains == 1> rd[kChains];
#pragma unroll
            for (uint32_t h = 0; h < kChains; ++h) {
                rd[h].start(area, 32 * (uint32_t)(fw[h] - 4 * bq) + (uint32_t)(p0[h] & 31), ok[h]);
            }
            auto entry = [&](uint32_t h) -> uint32_t {
                return stage_entry<kLong, kChains == 1>(rd[h], s_lut16, s_lut_len, s_lut_sym, lut_shift, K, max_len, s_first, s_count, s_base,
                                                        s_sorted, bad);
            };
            uint32_t ow[kChains * kChainWords];
#pragma unroll
            for (uint32_t q = 0; q < kChains * kChainWords; ++q) ow[q] = 0;  // (nothing flows from an earlier pass)
            uint32_t done[kChains];  // symbols of each chunk decoded into ow (whole rounds)
            bool all_full = true;
#pragma unroll
            for (uint32_t h = 0; h < kChains; ++h) all_full = all_full && ok[h] && s1[h] - s0[h] == S_eff;
            if (kChains > 1 && all_full && S_eff % R == 0) {
                // the usual case: both chunks whole, their codes decoded in turn
                const uint32_t nr = S_eff / R;
#pragma unroll
                for (uint32_t r = 0; r < kChainRounds; ++r) {
                    if (r < nr) {
                        uint32_t o4[kChains][kRoundWords];
#pragma unroll
                        for (uint32_t h = 0; h < kChains; ++h)
#pragma unroll
                            for (uint32_t q = 0; q < kRoundWords; ++q) o4[h][q] = 0;
#pragma unroll
                        for (uint32_t q = 0; q < R; ++q) {
#pragma unroll
                            for (uint32_t h = 0; h < kChains; ++h) o4[h][q >> 2] = put_sym<kLong ? 1 : 0>(entry(h), o4[h][q >> 2], q);
                            if ((q + 1) % SPR == 0 || q + 1 == R)
#pragma unroll
                                for (uint32_t h = 0; h < kChains; ++h) rd[h].refill();
                        }
#pragma unroll
                        for (uint32_t h = 0; h < kChains; ++h)
#pragma unroll
                            for (uint32_t q = 0; q < kRoundWords; ++q) ow[h * kChainWords + kRoundWords * r + q] = o4[h][q];
                    }
                }
#pragma unroll
                for (uint32_t h = 0; h < kChains; ++h) done[h] = nr * R;
            } else {
                // one chunk after the other: a block's short last chunk, a
                // chunk that failed its checks, or one chunk per lane
#pragma unroll
                for (uint32_t h = 0; h < kChains; ++h) {
                    done[h] = 0;
                    if (ok[h]) {
                        const uint32_t nfull = (s1[h] - s0[h]) / R;
#pragma unroll
                        for (uint32_t r = 0; r < kChainRounds; ++r) {
                            if (r < nfull) {
                                uint32_t o4[kRoundWords];
#pragma unroll
                                for (uint32_t q = 0; q < kRoundWords; ++q) o4[q] = 0;
#pragma unroll
                                for (uint32_t q = 0; q < R; ++q) {
                                    o4[q >> 2] = put_sym<kLong ? 1 : 0>(entry(h), o4[q >> 2], q);
                                    if ((q + 1) % SPR == 0 || q + 1 == R) rd[h].refill();
                                }
#pragma unroll
                                for (uint32_t q = 0; q < kRoundWords; ++q) ow[h * kChainWords + kRoundWords * r + q] = o4[q];
                            }
                        }
                        done[h] = nfull * R;
                        HC_G uint8_t *const dst = out + blk_start[h] + s0[h];
                        for (uint32_t q = done[h]; q < s1[h] - s0[h]; ++q) {  // the ragged end of a block's last chunk
                            dst[q] = (uint8_t)(entry(h) >> (kLong ? 8 : 0));
                            rd[h].refill();
                        }
                    }
                }
            }
            if (coalesce) {
                // all 64 lanes are here.  Each half of the wave in turn puts its
                // 128-byte lines into the area (lane stride 36 words: a 16-byte
                // write instruction covers all 64 banks), then the wave stores
                // them with lane l on 16 bytes 64u + l: every store instruction
                // writes a contiguous 1 KiB instead of touching 64 lines
                const uint64_t a0 = (uint64_t)(out + blk_start[0] + s0[0]);
                HC_G uint8_t *const base =
                    (HC_G uint8_t *)read_lane_u64(a0, 0);
                wave_lds_sync();  // the decode's reads of the area are done
#pragma unroll
                for (uint32_t half = 0; half < 2; ++half) {
                    if ((lane >> 5) == half) {
#pragma unroll
                        for (uint32_t r = 0; r < 8; ++r)
                            *(v4u *)(area + 36 * (lane & 31u) + 4 * r) = v4u{ow[4 * r], ow[4 * r + 1], ow[4 * r + 2], ow[4 * r + 3]};
                    }
                    wave_lds_sync();
#pragma unroll
                    for (uint32_t u = 0; u < 4; ++u) {
                        const uint32_t Q = 64 * u + lane;
                        *(HC_G v4u *)(base + 4096 * half + 16 * Q) = *(const v4u *)(area + 36 * (Q >> 3) + 4 * (Q & 7u));
                    }
                    wave_lds_sync();
                }
            }
            // each chunk's output (unless stored above): whole 16-byte pieces
            // from the registers, then (rounds of 8 symbols) a last 8-byte
            // piece; then its checks
#pragma unroll
            for (uint32_t h = 0; h < kChains; ++h) {
                if (ok[h] && !coalesce) {
                    HC_G uint8_t *const dst = out + blk_start[h] + s0[h];
                    const uint32_t k = done[h];
#pragma unroll
                    for (uint32_t r = 0; r < kChainSyms / 16; ++r)
                        if (16 * r + 16 <= k)
                            *(HC_G v4u *)(dst + 16 * r) = v4u{ow[h * kChainWords + 4 * r], ow[h * kChainWords + 4 * r + 1],
                                                              ow[h * kChainWords + 4 * r + 2], ow[h * kChainWords + 4 * r + 3]};
                    if (R == 8 && (k & 8u)) {
#pragma unroll
                        for (uint32_t r = 0; r < kChainSyms / 16; ++r)
                            if (16 * r + 8 == k)
                                *(HC_G v2u *)(dst + 16 * r) = v2u{ow[h * kChainWords + 4 * r], ow[h * kChainWords + 4 * r + 1]};
                    }
                }
                if (ok[h]) {
                    const uint64_t pos = 128 * bq + rd[h].position(area) - 32 * pw0[h];  // payload bits consumed
                    if (pos != p1[h]) report(err, HC_ERR_CORRUPT);
                    if (s1[h] == cnt[h] && (hdr[h] & 31u)) {
                        const uint32_t mask = (1u << (32 - (hdr[h] & 31u))) - 1u;
                        if (in32[pw0[h] + nwords[h] - 1] & mask) report(err, HC_ERR_CORRUPT);
                    }
                }
            }
            if (bad & kLutBadFlag) report(err, HC_ERR_CORRUPT);
        }
        wave_lds_sync();  // every read of this pass before the next pass's copy
        pending = pending && !take;
    }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_histogram(const JobList &jl, uint64_t units, uint64_t chunk, hipStream_t s)
{
    k_hist_zero<<<dim3(jl.count), kNumSym, 0, s>>>(jl);
    if (units) k_hist<<<dim3((uint32_t)units), kHistThreads, 0, s>>>(jl, chunk);
    return hipGetLastError();
}

hipError_t launch_put_jobs(const Job *jobs, uint32_t count, uint64_t total, Job *d_jobs, uint64_t *d_starts,
                           hipStream_t s)
{
    for (uint32_t first = 0; first < count; first += kJobsPerPut) {
        JobChunk c;
        c.first = first;
        c.count = count - first < kJobsPerPut ? count - first : kJobsPerPut;
        c.table_count = count;
        c.total = total;
        for (uint32_t k = 0; k < c.count; ++k) c.jobs[k] = jobs[first + k];
        k_put_jobs<<<1, kJobsPerPut, 0, s>>>(c, d_jobs, d_starts);
    }
    return hipGetLastError();
}

hipError_t launch_encode(const JobList &jl, uint64_t tiles, uint32_t B, uint32_t qpt, uint32_t max_len, uint32_t S,
                         void *scratch, uint32_t *err, hipStream_t s, uint32_t steps, bool complete8)
{
    if (tiles == 0) return hipSuccess;
    const uint32_t tpb = tiles_per_block(B, qpt);
    // the packing's LDS words (none for complete 8-bit codes: tiles are copied)
    // a multiple of 4: the packing clears the words 16 bytes at a time
    const uint32_t lds_words =
        complete8 ? 0u : (uint32_t)((((uint64_t)kTileSyms * qpt * max_len + 31ull) / 32ull + 2 + 3) & ~3ull);
    const uint32_t cpb = S ? (B + S - 1) / S : 1;
    uint32_t *tile_bits = static_cast<uint32_t *>(scratch);
    uint32_t *tile_pos = tile_bits + tiles;
    uint16_t *thread_bits = qpt >= 2 ? reinterpret_cast<uint16_t *>(tile_pos + tiles) : nullptr;
    const dim3 grid((uint32_t)tiles);
    const size_t lds = lds_words * 4;
    const bool packed = max_len <= (uint32_t)kPackedMaxLen;
    // 1. lengths (none for complete 8-bit codes: 8 bits a symbol)
    if (!(steps & kStepLengths) || complete8)
        ;
    else if (qpt == 4)
        k_count<4><<<grid, kTileThreads, 0, s>>>(jl, B, tpb, tile_bits, thread_bits, max_len, err);
    else if (qpt == 2)
        k_count<2><<<grid, kTileThreads, 0, s>>>(jl, B, tpb, tile_bits, thread_bits, max_len, err);
    else
        k_count<1><<<grid, kTileThreads, 0, s>>>(jl, B, tpb, tile_bits, thread_bits, max_len, err);
    // 2. offsets
    if (steps & kStepOffsets)
        k_offsets<<<dim3(jl.count), kOffThreads, 0, s>>>(jl, B, tpb, tile_bits, tile_pos,
                                                         complete8 ? kTileSyms * qpt : 0u, err);
    // 3. packing
#define HC_ENC(P, F, Q) k_encode<P, F, Q><<<grid, kTileThreads, lds, s>>>(jl, B, tpb, tile_pos, thread_bits, S, cpb, lds_words, max_len, complete8 ? 1u : 0u, err)
    if (!(steps & kStepPack)) {
    } else if (!packed) {
        HC_ENC(false, 1, 1);
    } else {
        // FPS codes between accumulator flushes: FPS * max_len <= 32
        const uint32_t fps = max_len <= 8 ? 4 : max_len <= 10 ? 3 : max_len <= 16 ? 2 : 1;
        switch (fps * 8 + qpt) {
        case 4 * 8 + 4: HC_ENC(true, 4, 4); break;
        case 4 * 8 + 2: HC_ENC(true, 4, 2); break;
        case 4 * 8 + 1: HC_ENC(true, 4, 1); break;
        case 3 * 8 + 4: HC_ENC(true, 3, 4); break;
        case 3 * 8 + 2: HC_ENC(true, 3, 2); break;
        case 3 * 8 + 1: HC_ENC(true, 3, 1); break;
        case 2 * 8 + 4: HC_ENC(true, 2, 4); break;
        case 2 * 8 + 2: HC_ENC(true, 2, 2); break;
        case 2 * 8 + 1: HC_ENC(true, 2, 1); break;
        case 1 * 8 + 2: HC_ENC(true, 1, 2); break;
        case 1 * 8 + 1: HC_ENC(true, 1, 1); break;
        default: return hipErrorInvalidValue;  // encode_qpt never pairs these
        }
    }
#undef HC_ENC
    return hipGetLastError();
}

hipError_t launch_walk(const uint8_t *in, uint64_t in_bytes, uint64_t nb, uint64_t *block_off,
                       uint32_t *err, hipStream_t s)
{
    k_walk<<<1, 64, 0, s>>>(reinterpret_cast<const uint32_t *>(in), in_bytes, nb, block_off, err);
    return hipGetLastError();
}

hipError_t launch_encode_empty(uint64_t *block_off, hipStream_t s)
{
    k_fill_u64<<<1, 64, 0, s>>>(block_off, 1, 0);
    return hipGetLastError();
}

hipError_t launch_decode_sync(const JobList &jl, uint64_t blocks, uint32_t B, uint32_t max_len, uint32_t *err,
                              hipStream_t s)
{
    if (blocks == 0) return hipSuccess;
    // the longest payload a block can have (B codes of max_len bits), up to the LDS copy's limit
    const uint64_t need = ((uint64_t)B * max_len + 31) / 32;
    const uint32_t stage = (uint32_t)(need < kSyncStageWords ? need : kSyncStageWords);
    k_decode_sync<<<dim3((uint32_t)blocks), kSyncThreads, (size_t)stage * 4, s>>>(jl, B, stage, max_len, err);
    return hipGetLastError();
}

hipError_t launch_decode(const JobList &jl, uint64_t groups, uint32_t B, uint32_t max_len, uint32_t S,
                         bool with_index, uint32_t *err, hipStream_t s, bool complete8)
{
    if (groups == 0) return hipSuccess;
    const uint32_t S_eff = decode_chunk(B, S, with_index, complete8);
    const uint32_t cpb = (B + S_eff - 1) / S_eff;
    const dim3 grid((uint32_t)groups);
    if (complete8) {  // every job a complete 8-bit code: the copy form, no ring, no table
        k_decode_ring<16, 4, false, true><<<grid, kDecThreads, 0, s>>>(jl, B, S_eff, cpb, max_len, err);
        return hipGetLastError();
    }
    // the table has 2^lut_bits entries, lut_bits = min(max_len, kLutBits) of the longest code
    const size_t lut = (size_t)2 << (max_len < (uint32_t)kLutBits ? max_len : (uint32_t)kLutBits);
    if (with_index && S <= kStageMaxS && max_len <= (uint32_t)kPackedMaxLen) {
        // wave-staged chunks; the table sized for the longest code's lut_bits;
        // two chunks per lane up to 64 symbols (groups of 128 lanes)
#define HC_STG(R, P, L, T)                                                                                       \
    do {                                                                                                          \
        if (S <= kStageMaxS / 2)                                                                                  \
            k_decode_stage<R, P, L, T, 2><<<grid, kDecThreads / 2, 0, s>>>(jl, B, S_eff, cpb, max_len, err);               \
        else                                                                                                      \
            k_decode_stage<R, P, L, T, 1><<<grid, kDecThreads, 0, s>>>(jl, B, S_eff, cpb, max_len, err);                   \
    } while (0)
        if (max_len <= 8)
            HC_STG(16, 4, false, 8);
        else if (max_len <= 10)
            HC_STG(16, 3, false, 10);
        else if (max_len <= (uint32_t)kLutBits)
            HC_STG(16, 2, false, 12);
        else if (max_len <= 16)
            HC_STG(16, 2, true, 12);
        else
            HC_STG(8, 1, true, 12);
#undef HC_STG
        return hipGetLastError();
    }
    // a round of R symbols of <= 32 * 16 / R bits stays within one ring half (16 words)
    if (max_len <= 8)
        k_decode_ring<16, 4, false><<<grid, kDecThreads, lut, s>>>(jl, B, S_eff, cpb, max_len, err);
    else if (max_len <= 10)
        k_decode_ring<16, 3, false><<<grid, kDecThreads, lut, s>>>(jl, B, S_eff, cpb, max_len, err);
    else if (max_len <= (uint32_t)kLutBits)
        k_decode_ring<16, 2, false><<<grid, kDecThreads, lut, s>>>(jl, B, S_eff, cpb, max_len, err);
    else if (max_len <= 16)
        k_decode_ring<16, 2, true><<<grid, kDecThreads, lut, s>>>(jl, B, S_eff, cpb, max_len, err);
    else if (max_len <= (uint32_t)kPackedMaxLen)  // 8 symbols of <= 24 bits: 6 words
        k_decode_ring<8, 1, true><<<grid, kDecThreads, lut, s>>>(jl, B, S_eff, cpb, max_len, err);
    else
        k_decode<<<grid, kDecThreads, 0, s>>>(jl, B, S_eff, cpb, err);
    return hipGetLastError();
}

}  // namespace hc
