// HIP kernels for gfx950 (CDNA4, wave64) of the block-decomposed Huffman codec.
//
//   k_hist         symbol counts (paper section 2) with LDS-privatised
//                  sub-histograms, one replica per lane of a wavefront
//   k_tile_bits    length pass (section 2.1): payload bits of each tile of
//                  4096 symbols (a tile never crosses a block boundary)
//   k_block_sums   per block: tile bit prefixes, block bit count, block bytes
//   k_scan_*       exclusive scan of block bytes -> block offsets (section 2.1)
//   k_pack         bit packing (section 2.1, Fig. 3-4): each tile's code words
//                  are OR-ed into LDS words at their final bit alignment and
//                  stored, coalesced, at the block's offset in the stream
//   k_walk         offset table rebuilt from the length delimiters
//   k_decode       table decode (sections 2.1 and 3.2): one lane per block, or
//                  per chunk of S symbols when a sub-block index is given
#include <hip/hip_runtime.h>

#include "hc_internal.h"
#include "hc_kernels.h"

namespace hc {

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ void report(uint32_t *err, uint32_t code)
{
    if (err) atomicCAS(err, 0u, code);
}

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
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
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

// ---------------------------------------------------------------- histogram
// Each work-group counts a contiguous chunk into 64 LDS sub-histograms laid
// out bin-major (sub-histogram r of bin v at v*64 + r); lane r of every wave
// adds into sub-histogram r, so the 64 lanes of one LDS atomic always touch 64
// consecutive words whatever the data (no bank conflicts, no same-address
// serialisation on skewed inputs).  The group then folds the 64 copies and adds
// its counts to the global u64 histogram.
__global__ __launch_bounds__(kHistThreads) void k_hist(const uint8_t *__restrict__ in, uint64_t n,
                                                       uint64_t chunk,
                                                       unsigned long long *__restrict__ hist)
{
    __shared__ uint32_t sh[kNumSym * 64];
    for (int k = threadIdx.x; k < kNumSym * 64; k += kHistThreads) sh[k] = 0;
    __syncthreads();

    const uint32_t lane = threadIdx.x & 63;
    const uint64_t beg = (uint64_t)blockIdx.x * chunk;
    const uint64_t end = beg + chunk < n ? beg + chunk : n;
    const uint64_t nvec = (end - beg) >> 4;
    const uint4 *p = reinterpret_cast<const uint4 *>(in + beg);

    auto add_word = [&](uint32_t w) {
        atomicAdd(&sh[((w)&255u) * 64 + lane], 1u);
        atomicAdd(&sh[((w >> 8) & 255u) * 64 + lane], 1u);
        atomicAdd(&sh[((w >> 16) & 255u) * 64 + lane], 1u);
        atomicAdd(&sh[(w >> 24) * 64 + lane], 1u);
    };
    auto add_vec = [&](uint4 q) {
        add_word(q.x);
        add_word(q.y);
        add_word(q.z);
        add_word(q.w);
    };

    uint64_t v = threadIdx.x;
    for (; v + 3 * kHistThreads < nvec; v += 4 * kHistThreads) {
        uint4 a = p[v];
        uint4 b = p[v + kHistThreads];
        uint4 c = p[v + 2 * kHistThreads];
        uint4 d = p[v + 3 * kHistThreads];
        add_vec(a);
        add_vec(b);
        add_vec(c);
        add_vec(d);
    }
    for (; v < nvec; v += kHistThreads) add_vec(p[v]);
    for (uint64_t j = beg + (nvec << 4) + threadIdx.x; j < end; j += kHistThreads)
        atomicAdd(&sh[(uint32_t)in[j] * 64 + lane], 1u);
    __syncthreads();

    if (threadIdx.x < kNumSym) {
        const uint32_t b = threadIdx.x;
        uint64_t s = 0;
#pragma unroll 8
        for (uint32_t r = 0; r < 64; ++r) s += sh[b * 64 + ((r + b) & 63u)];  // rotated: no conflicts
        if (s) atomicAdd(&hist[b], (unsigned long long)s);
    }
}

// ---------------------------------------------------------------- tiles
struct Tile {
    uint64_t blk;       // block index
    uint32_t j;         // tile index inside the block
    uint64_t blk_start; // first symbol of the block
    uint32_t cnt;       // symbols in the block
    uint32_t ts, te;    // symbol range of the tile, relative to the block
};

__device__ __forceinline__ Tile tile_of(const TileGeom &g, uint64_t t)
{
    Tile r;
    r.blk = t / g.tpb;
    r.j = (uint32_t)(t - r.blk * g.tpb);
    r.blk_start = r.blk * (uint64_t)g.B;
    const uint64_t left = g.n - r.blk_start;
    r.cnt = (uint32_t)(left < g.B ? left : g.B);
    r.ts = r.j * kTileSyms;
    const uint32_t e = r.ts + kTileSyms;
    r.te = e < r.cnt ? e : r.cnt;
    if (r.ts > r.te) r.ts = r.te;  // empty tile past the end of a short last block
    return r;
}

// Loads the (up to) 16 symbols of this thread; returns how many there are.
__device__ __forceinline__ uint32_t load16(const uint8_t *__restrict__ in, const Tile &tl, uint32_t s,
                                           uint32_t w[4])
{
    w[0] = w[1] = w[2] = w[3] = 0;
    if (s >= tl.te) return 0;
    const uint8_t *src = in + tl.blk_start + s;
    if (s + 16 <= tl.te) {
        uint4 q = *reinterpret_cast<const uint4 *>(src);
        w[0] = q.x;
        w[1] = q.y;
        w[2] = q.z;
        w[3] = q.w;
        return 16;
    }
    const uint32_t m = tl.te - s;
    for (uint32_t k = 0; k < m; ++k) w[k >> 2] |= (uint32_t)src[k] << (8 * (k & 3));
    return m;
}

__device__ __forceinline__ uint32_t sym_at(const uint32_t w[4], uint32_t k)
{
    return (w[k >> 2] >> (8 * (k & 3))) & 255u;
}

// Length pass: bits of every tile.
__global__ __launch_bounds__(kTileThreads) void k_tile_bits(const uint8_t *__restrict__ in, TileGeom g,
                                                            const DevTables *__restrict__ tb,
                                                            uint32_t *__restrict__ tile_bits,
                                                            uint32_t *err)
{
    __shared__ uint32_t slen[kNumSym];
    __shared__ uint32_t sred[kTileThreads / 64];
    slen[threadIdx.x] = tb->enc_len[threadIdx.x];
    __syncthreads();

    const uint64_t t = blockIdx.x;
    const Tile tl = tile_of(g, t);
    uint32_t w[4];
    const uint32_t m = load16(in, tl, tl.ts + kSymPerThread * threadIdx.x, w);
    uint32_t bits = 0;
    bool absent = false;
#pragma unroll
    for (uint32_t k = 0; k < 16; ++k) {
        if (k < m) {
            const uint32_t L = slen[sym_at(w, k)];
            absent |= (L == 0);
            bits += L;
        }
    }
    if (absent) report(err, HC_ERR_SYMBOL_ABSENT);
    bits = wave_sum(bits);
    if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = bits;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < kTileThreads / 64; ++k) s += sred[k];
        tile_bits[t] = s;
    }
}

// Per block: bit position of each tile inside the block, the block's bit count
// and its size in bytes (header + payload words), the latter into 'bytes'.
__global__ void k_block_sums(TileGeom g, const uint32_t *__restrict__ tile_bits,
                             uint32_t *__restrict__ tile_pos, uint32_t *__restrict__ block_bits,
                             uint64_t *__restrict__ bytes, uint32_t *err)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.nb) return;
    uint64_t s = 0;
    for (uint32_t j = 0; j < g.tpb; ++j) {
        tile_pos[i * g.tpb + j] = (uint32_t)s;
        s += tile_bits[i * g.tpb + j];
    }
    if (s > 0xFFFFFFFFull) report(err, HC_ERR_BLOCK_OVERFLOW);
    block_bits[i] = (uint32_t)s;
    bytes[i] = 4 + 4 * ((s + 31) / 32);
}

// ---------------------------------------------------------------- scan
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint64_t *__restrict__ v,
                                                              uint64_t count,
                                                              uint64_t *__restrict__ partial)
{
    __shared__ uint64_t sred[kScanThreads / 64];
    const uint64_t base = (uint64_t)blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * kScanItems;
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < count) s += v[base + k];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
#pragma unroll
        for (int k = 0; k < kScanThreads / 64; ++k) t += sred[k];
        partial[blockIdx.x] = t;
    }
}

// One work-group: exclusive scan of the chunk sums, in place; total -> *total.
__global__ __launch_bounds__(kScanThreads) void k_scan_partials(uint64_t *__restrict__ partial,
                                                                uint64_t nchunks,
                                                                uint64_t *__restrict__ total)
{
    __shared__ uint64_t scratch[kScanThreads / 64];
    uint64_t carry = 0;
    for (uint64_t base = 0; base < nchunks; base += kScanChunk) {
        const uint64_t b = base + (uint64_t)threadIdx.x * kScanItems;
        uint64_t item[kScanItems];
        uint64_t s = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            item[k] = (b + k < nchunks) ? partial[b + k] : 0;
            s += item[k];
        }
        uint64_t all;
        uint64_t run = carry + group_exclusive_scan<uint64_t, kScanThreads>(s, scratch, &all);
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            if (b + k < nchunks) partial[b + k] = run;
            run += item[k];
        }
        carry += all;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(uint64_t *__restrict__ v, uint64_t count,
                                                            const uint64_t *__restrict__ partial)
{
    __shared__ uint64_t scratch[kScanThreads / 64];
    const uint64_t b = (uint64_t)blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * kScanItems;
    uint64_t item[kScanItems];
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        item[k] = (b + k < count) ? v[b + k] : 0;
        s += item[k];
    }
    uint64_t all;
    uint64_t run = partial[blockIdx.x] + group_exclusive_scan<uint64_t, kScanThreads>(s, scratch, &all);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (b + k < count) v[b + k] = run;
        run += item[k];
    }
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

template <bool kPacked>
__global__ __launch_bounds__(kTileThreads) void k_pack(
    const uint8_t *__restrict__ in, TileGeom g, const DevTables *__restrict__ tb,
    const uint32_t *__restrict__ tile_bits, const uint32_t *__restrict__ tile_pos,
    const uint32_t *__restrict__ block_bits, const uint64_t *__restrict__ block_off,
    uint32_t *__restrict__ out32, uint32_t *__restrict__ sub_idx, uint32_t S, uint32_t cpb,
    uint32_t lds_words)
{
    extern __shared__ uint32_t words[];  // lds_words words: the tile's payload at its bit alignment
    __shared__ uint32_t s_packed[kNumSym];
    __shared__ uint64_t s_code[kPacked ? 1 : kNumSym];
    __shared__ uint32_t s_len[kPacked ? 1 : kNumSym];
    __shared__ uint32_t s_scan[kTileThreads / 64];
    __shared__ uint32_t s_next[32];
    __shared__ uint32_t s_fill;

    const uint64_t t = blockIdx.x;
    const Tile tl = tile_of(g, t);
    if (tl.ts >= tl.te) return;  // empty tile (uniform over the group)
    const uint32_t tid = threadIdx.x;

    if (kPacked) {
        s_packed[tid] = tb->enc_packed[tid];
    } else {
        s_code[tid] = tb->enc_code[tid];
        s_len[tid] = tb->enc_len[tid];
    }
    const bool last_tile = tl.te == tl.cnt;
    if (tid < 32) {  // the symbols just past the tile, for the word it shares with the next tile
        const uint32_t k = tl.te + tid;
        s_next[tid] = (!last_tile && k < tl.cnt) ? in[tl.blk_start + k] : 0u;
    }
    for (uint32_t k = tid; k < lds_words; k += kTileThreads) words[k] = 0;

    const uint32_t s = tl.ts + kSymPerThread * tid;
    uint32_t w[4];
    const uint32_t m = load16(in, tl, s, w);
    __syncthreads();

    uint32_t bits = 0;
#pragma unroll
    for (uint32_t k = 0; k < 16; ++k) {
        if (k < m) bits += kPacked ? (s_packed[sym_at(w, k)] & 255u) : s_len[sym_at(w, k)];
    }
    uint32_t tile_total;
    const uint32_t q = group_exclusive_scan<uint32_t, kTileThreads>(bits, s_scan, &tile_total);

    const uint32_t P = tile_pos[t];  // bit position of the tile inside the block's payload
    const uint32_t a = P & 31u;
    {
        const uint32_t start = a + q;
        uint32_t widx = start >> 5;
        uint32_t nacc = start & 31u;  // leading zero bits keep the word aligned
        uint64_t acc = 0;
#pragma unroll
        for (uint32_t k = 0; k < 16; ++k) {
            if (k < m) {
                const uint32_t v = sym_at(w, k);
                if (kPacked) {
                    const uint32_t e = s_packed[v];
                    put_bits(acc, nacc, widx, e >> 8, e & 255u, words);
                } else {
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

    // Word ownership: a stream word is written by the tile that holds its first
    // bit.  If the tile's last word continues into the next tile of the block,
    // this tile completes it from the first symbols of that tile (which then
    // skips the word); at the end of a block the remaining bits are zero pad.
    const uint32_t e_bits = a + tile_total;     // end of the tile, in LDS bits
    const uint32_t k_first = (a == 0) ? 0u : 1u;
    // tile_total is 0 only if a symbol had no code (already reported): store nothing
    const uint32_t k_last = tile_total ? (e_bits - 1) >> 5 : 0u;
    const uint32_t k_end = tile_total ? k_last + 1 : 0u;
    if (tid == 0) {
        uint64_t fill = 0;
        if (!last_tile && (e_bits & 31u)) {
            const uint32_t need = 32 - (e_bits & 31u);
            const uint32_t avail = tl.cnt - tl.te < 32 ? tl.cnt - tl.te : 32;
            uint32_t got = 0;
            for (uint32_t k = 0; k < avail && got < need; ++k) {
                const uint32_t v = s_next[k];
                uint32_t L;
                uint64_t c;
                if (kPacked) {
                    L = s_packed[v] & 255u;
                    c = s_packed[v] >> 8;
                } else {
                    L = s_len[v];
                    c = s_code[v];
                }
                const uint32_t r = need - got;
                if (L >= r) {
                    fill = (fill << r) | (c >> (L - r));
                    got = need;
                } else {
                    fill = (fill << L) | c;
                    got += L;
                }
            }
            fill <<= (need - got);
        }
        s_fill = (uint32_t)fill;
    }
    __syncthreads();  // all code words are in LDS, s_fill is set

    const uint64_t off = block_off[tl.blk];
    uint32_t *payload = out32 + (off >> 2) + 1 + (P >> 5);
    for (uint32_t k = k_first + tid; k < k_end; k += kTileThreads)
        payload[k] = (k == k_last) ? (words[k] | s_fill) : words[k];

    if (tl.j == 0 && tid == 0) out32[off >> 2] = block_bits[tl.blk];
    if (sub_idx) {
        if (m > 0 && (s % S) == 0) sub_idx[tl.blk * cpb + s / S] = P + q;
        if (last_tile && tid == 0) {
            const uint32_t bb = block_bits[tl.blk];
            for (uint32_t c = (tl.cnt + S - 1) / S; c < cpb; ++c) sub_idx[tl.blk * cpb + c] = bb;
        }
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
__device__ __forceinline__ uint32_t ld_word(const uint32_t *__restrict__ payload, uint32_t nwords,
                                            uint32_t w)
{
    return w < nwords ? payload[w] : 0u;
}

// 64 payload bits starting at bit p (bits past the payload read as 0).
__device__ __forceinline__ uint64_t window64(const uint32_t *__restrict__ payload, uint32_t nwords,
                                             uint64_t p)
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

    __device__ __forceinline__ void seek(const uint32_t *payload, uint32_t nwords, uint64_t p)
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
__device__ __forceinline__ uint32_t decode_one(BitReader &br, const uint32_t *__restrict__ payload,
                                               uint32_t nwords, const uint16_t *lut, uint32_t K,
                                               uint32_t max_len, const uint64_t *first,
                                               const uint32_t *count, const uint32_t *base,
                                               const uint32_t *sorted, bool &bad)
{
    if (br.nbits < 32) {
        br.buf |= (uint64_t)ld_word(payload, nwords, br.wi) << (32 - br.nbits);
        br.nbits += 32;
        br.wi += 1;
    }
    const uint32_t e = lut[br.buf >> (64 - K)];
    const uint32_t L = e >> 8;
    if (L != 0 && e != kLutInvalid) {
        br.buf <<= L;
        br.nbits -= L;
        return e & 255u;
    }
    if (e == kLutInvalid) {
        bad = true;
        return 0;
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

__global__ __launch_bounds__(kDecThreads) void k_decode(
    const uint32_t *__restrict__ in32, uint64_t in_bytes, uint64_t n, uint32_t B, uint64_t nb,
    const DevTables *__restrict__ tb, const uint64_t *__restrict__ off,
    const uint32_t *__restrict__ sub_idx, uint32_t S_eff, uint32_t cpb, uint8_t *__restrict__ out,
    uint32_t *err)
{
    __shared__ uint16_t s_lut[1 << kLutBits];
    __shared__ uint64_t s_first[kMaxLen + 1];
    __shared__ uint32_t s_count[kMaxLen + 1];
    __shared__ uint32_t s_base[kMaxLen + 1];
    __shared__ uint32_t s_sorted[kNumSym];

    const uint32_t tid = threadIdx.x;
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

    const uint64_t g = (uint64_t)blockIdx.x * kDecThreads + tid;
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
    const uint32_t *payload = in32 + (o >> 2) + 1;
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
    uint8_t *dst = out + blk_start;
    uint32_t k = s0;
    for (; k + 16 <= s1 && !bad; k += 16) {
        uint32_t o4[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (uint32_t q = 0; q < 16; ++q) {
            const uint32_t sym = decode_one(br, payload, nwords, s_lut, K, max_len, s_first, s_count,
                                            s_base, s_sorted, bad);
            o4[q >> 2] |= sym << (8 * (q & 3));
        }
        *reinterpret_cast<uint4 *>(dst + k) = make_uint4(o4[0], o4[1], o4[2], o4[3]);
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

// ---------------------------------------------------------------- launchers
static inline uint64_t align16(uint64_t x) { return (x + 15) & ~uint64_t(15); }

uint64_t encode_ws_bytes(const TileGeom &g)
{
    const uint64_t ntiles = g.nb * g.tpb;
    const uint64_t nchunks = (g.nb + kScanChunk - 1) / kScanChunk;
    return align16(4 * ntiles) * 2 + align16(4 * g.nb) + align16(8 * (nchunks ? nchunks : 1));
}

EncodeWs carve_encode_ws(void *ws, const TileGeom &g)
{
    const uint64_t ntiles = g.nb * g.tpb;
    char *p = static_cast<char *>(ws);
    EncodeWs w;
    w.tile_bits = reinterpret_cast<uint32_t *>(p);
    p += align16(4 * ntiles);
    w.tile_pos = reinterpret_cast<uint32_t *>(p);
    p += align16(4 * ntiles);
    w.block_bits = reinterpret_cast<uint32_t *>(p);
    p += align16(4 * g.nb);
    w.partial = reinterpret_cast<uint64_t *>(p);
    return w;
}

hipError_t launch_histogram(const uint8_t *in, uint64_t n, uint64_t *hist, hipStream_t s)
{
    k_fill_u64<<<1, kNumSym, 0, s>>>(hist, kNumSym, 0);
    if (n == 0) return hipGetLastError();
    uint64_t chunk = (n + kHistTargetGroups - 1) / kHistTargetGroups;
    chunk = (chunk + 15) & ~uint64_t(15);
    if (chunk < kHistMinChunk) chunk = kHistMinChunk;
    if (chunk > (1ull << 30)) chunk = 1ull << 30;  // keeps every LDS counter below 2^32
    const uint64_t groups = (n + chunk - 1) / chunk;
    k_hist<<<dim3((uint32_t)groups), kHistThreads, 0, s>>>(in, n, chunk,
                                                           reinterpret_cast<unsigned long long *>(hist));
    return hipGetLastError();
}

hipError_t launch_encode(const uint8_t *in, const TileGeom &g, const DevTables *tb, uint32_t max_len,
                         uint8_t *out, uint64_t *block_off, uint32_t *sub_idx, uint32_t S,
                         const EncodeWs &ws, uint32_t *err, hipStream_t s)
{
    if (g.n == 0) {
        k_fill_u64<<<1, 64, 0, s>>>(block_off, 1, 0);
        return hipGetLastError();
    }
    const uint64_t ntiles = g.nb * g.tpb;
    const uint64_t nchunks = (g.nb + kScanChunk - 1) / kScanChunk;
    k_tile_bits<<<dim3((uint32_t)ntiles), kTileThreads, 0, s>>>(in, g, tb, ws.tile_bits, err);
    k_block_sums<<<dim3((uint32_t)((g.nb + 255) / 256)), 256, 0, s>>>(g, ws.tile_bits, ws.tile_pos,
                                                                      ws.block_bits, block_off, err);
    k_scan_reduce<<<dim3((uint32_t)nchunks), kScanThreads, 0, s>>>(block_off, g.nb, ws.partial);
    k_scan_partials<<<1, kScanThreads, 0, s>>>(ws.partial, nchunks, block_off + g.nb);
    k_scan_down<<<dim3((uint32_t)nchunks), kScanThreads, 0, s>>>(block_off, g.nb, ws.partial);
    const uint32_t lds_words = (uint32_t)((31ull + (uint64_t)kTileSyms * max_len + 31ull) / 32ull + 1);
    const uint32_t cpb = S ? (g.B + S - 1) / S : 1;
    uint32_t *out32 = reinterpret_cast<uint32_t *>(out);
    if (max_len <= (uint32_t)kPackedMaxLen)
        k_pack<true><<<dim3((uint32_t)ntiles), kTileThreads, lds_words * 4, s>>>(
            in, g, tb, ws.tile_bits, ws.tile_pos, ws.block_bits, block_off, out32, sub_idx, S, cpb,
            lds_words);
    else
        k_pack<false><<<dim3((uint32_t)ntiles), kTileThreads, lds_words * 4, s>>>(
            in, g, tb, ws.tile_bits, ws.tile_pos, ws.block_bits, block_off, out32, sub_idx, S, cpb,
            lds_words);
    return hipGetLastError();
}

hipError_t launch_walk(const uint8_t *in, uint64_t in_bytes, uint64_t nb, uint64_t *block_off,
                       uint32_t *err, hipStream_t s)
{
    k_walk<<<1, 64, 0, s>>>(reinterpret_cast<const uint32_t *>(in), in_bytes, nb, block_off, err);
    return hipGetLastError();
}

hipError_t launch_decode(const uint8_t *in, uint64_t in_bytes, uint64_t n, uint32_t B, const DevTables *tb,
                         const uint64_t *block_off, const uint32_t *sub_idx, uint32_t S, uint8_t *out,
                         uint32_t *err, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const uint64_t nb = (n + B - 1) / B;
    const uint32_t S_eff = sub_idx ? S : B;
    const uint32_t cpb = sub_idx ? (B + S - 1) / S : 1;
    const uint64_t lanes = nb * cpb;
    const uint64_t groups = (lanes + kDecThreads - 1) / kDecThreads;
    k_decode<<<dim3((uint32_t)groups), kDecThreads, 0, s>>>(reinterpret_cast<const uint32_t *>(in),
                                                           in_bytes, n, B, nb, tb, block_off, sub_idx,
                                                           S_eff, cpb, out, err);
    return hipGetLastError();
}

}  // namespace hc
