// Library-internal definitions shared by the host glue and the kernels.
#pragma once

#include <stdint.h>

#include "hc.h"

namespace hc {

constexpr int kNumSym = 256;
constexpr int kMaxLen = 64;
constexpr int kLutBits = 12;  // first-level decode table: 4096 entries
// Decode table entry: (symbol << 8) | len for a code of len <= lut_bits bits;
// kLutLong if the prefix starts a longer code; kLutInvalid if no code starts
// with it: flag bit 7 in the length byte, and a shift of 1 in its low 6 bits
// (a decoder may shift by the entry's low 6 bits without a test; bit 7 then
// marks the stream corrupt).
constexpr uint16_t kLutLong = 0;
constexpr uint16_t kLutInvalid = 0x0081;
constexpr uint32_t kLutBadFlag = 0x80;
constexpr int kPackedMaxLen = 24;        // codes up to 24 bits fit (code << 8 | len) in a u32

// Device-resident tables of one codebook (one contiguous allocation).
struct DevTables {
    uint32_t enc_packed[kNumSym];  // (code << 8) | len, valid when max_len <= kPackedMaxLen
    uint64_t enc_code[kNumSym];    // right-aligned canonical code values
    uint32_t enc_len[kNumSym];     // code lengths, 0 = no code
    alignas(16) uint32_t len4[kNumSym / 4];  // the same lengths, four per word: symbol 4i + j in byte j of word i
    uint16_t lut[1 << kLutBits];   // next lut_bits bits -> (symbol << 8) | len
    uint64_t first[kMaxLen + 1];   // first canonical code value of each length
    uint32_t count[kMaxLen + 1];   // number of codes of each length
    uint32_t base[kMaxLen + 1];    // position in 'sorted' of the first code of each length
    uint32_t sorted[kNumSym];      // symbols in canonical order (length, value)
    uint32_t max_len;
    uint32_t nsym;
    uint32_t lut_bits;             // min(max_len, kLutBits), at least 1
    uint32_t fixed_len;            // L if every code has length L, else 0
};

// Fills the device tables for a (validated) host codebook.
void build_dev_tables(const hc_codebook &cb, DevTables *t);

// Kraft check and canonical assignment shared by the two codebook constructors.
hc_status canonical_from_lengths(const uint8_t *len, hc_codebook *out);

// hc_encode_blocks with its workspace given as a device address and size:
// the caller-workspace entry point and the allocation-free one both end here.
hc_status encode_blocks_ws(const uint8_t *d_in, uint64_t n, uint32_t block_size, hc_cb_handle cb, uint8_t *d_out,
                           uint64_t out_cap, uint64_t *d_block_off, uint32_t *d_sub_idx, uint32_t sub_block,
                           void *d_ws, uint64_t ws_bytes, uint32_t *d_err, void *stream);

}  // namespace hc

struct hc_cb_dev_s {
    hc_codebook host;
    hc::DevTables *d_tables;  // device copy read by the kernels
    hc::DevTables *staging;   // pinned host staging area for updates
    void *copy_done;          // hipEvent_t recorded after the last update copy
    int device;
    int in_set;               // owned by a codebook set (its tables live in the set's arrays)
};

struct hc_cbset_s {
    uint32_t count;
    hc_cb_dev_s *handles;     // count handles pointing into the arrays below
    hc::DevTables *d_tables;  // count tables, contiguous on the device
    hc::DevTables *staging;   // count tables, contiguous in pinned host memory
    void *copy_done;          // hipEvent_t recorded after the last build copy
};
