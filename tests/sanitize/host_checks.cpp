// Host-side checks run under AddressSanitizer and UndefinedBehaviorSanitizer
// (built with g++/gcc for the CPU only by tests/test_sanitizers.py): the
// oracle's C, the library's code construction and decode-table build, and the
// argument checks and job-table logic of every entry point, on random and
// edge-case inputs.  Any sanitizer report aborts the program; a mismatch
// between the oracle's and the library's code lengths exits with status 1.
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "hc.h"
#include "hc_internal.h"

extern "C" {
// the oracle (oracle/hc_oracle.c), test infrastructure linked into this driver
void or_histogram(const uint8_t *x, uint64_t n, uint64_t hist[256]);
int or_code_lengths(const uint64_t hist[256], uint8_t len[256]);
int or_canonical_codes(const uint8_t len[256], uint64_t code[256]);
uint64_t or_encoded_size(const uint8_t *x, uint64_t n, uint64_t B, const uint8_t len[256]);
int or_encode(const uint8_t *x, uint64_t n, uint64_t B, const uint8_t len[256], const uint64_t code[256],
              uint8_t *out, uint64_t out_cap, uint64_t *offsets, uint64_t *bits);
int or_walk(const uint8_t *in, uint64_t in_bytes, uint64_t nb, uint64_t *offsets);
int or_decode(const uint8_t *in, uint64_t in_bytes, uint64_t n, uint64_t B, const uint8_t len[256], uint8_t *out);
}

namespace {

uint64_t g_state = 0x1107152500000001ull;
uint64_t next_u64()
{  // SplitMix64 (Steele, Lea, Flood 2014)
    uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
uint64_t below(uint64_t m) { return m ? next_u64() % m : 0; }

int g_fail = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            g_fail = 1;                                                   \
        }                                                                 \
    } while (0)

void random_hist(uint64_t h[256])
{
    memset(h, 0, 256 * sizeof(uint64_t));
    switch (below(6)) {
    case 0:  // sparse small counts, many ties
        for (int k = 0; k < 1 + (int)below(40); ++k) h[below(256)] += 1 + below(4);
        break;
    case 1:  // dense random
        for (int v = 0; v < 256; ++v) h[v] = below(1000);
        break;
    case 2:  // Fibonacci weights: the deepest trees
    {
        const int m = 2 + (int)below(60);
        uint64_t a = 1, b = 1;
        for (int k = 0; k < m; ++k) {
            h[(k * 37) & 255] = a;
            const uint64_t c = a + b;
            a = b;
            b = c;
        }
        break;
    }
    case 3:  // one symbol, or none
        if (below(2)) h[below(256)] = 1 + below(1u << 20);
        break;
    case 4:  // huge counts whose sum still fits 64 bits
        for (int v = 0; v < 256; ++v) h[v] = below(1ull << 55);
        break;
    default:  // skewed
        h[below(256)] = 1 + below(1u << 24);
        for (int k = 0; k < 200; ++k) h[below(256)] += below(3);
    }
}

void check_codebooks()
{
    for (int it = 0; it < 20000; ++it) {
        uint64_t h[256];
        random_hist(h);
        uint8_t L_or[256];
        const int st_or = or_code_lengths(h, L_or);
        hc_codebook cb;
        const hc_status st = hc_build_codebook(h, &cb);
        if (st_or == 0) {
            CHECK(st == HC_OK);
            if (st != HC_OK) continue;
            CHECK(memcmp(cb.len, L_or, 256) == 0);
            uint64_t C_or[256];
            if (or_canonical_codes(L_or, C_or) == 0) CHECK(memcmp(cb.code, C_or, sizeof(C_or)) == 0);
            if (cb.max_len > 0) {
                static hc::DevTables t;
                hc::build_dev_tables(cb, &t);
                CHECK(t.max_len == cb.max_len && t.nsym == cb.nsym);
            }
        } else {
            CHECK(st != HC_OK);
        }
    }
    // lengths given directly: valid, over-full and over-long sets
    for (int it = 0; it < 5000; ++it) {
        uint8_t L[256] = {0};
        const int m = (int)below(257);
        for (int k = 0; k < m; ++k) L[below(256)] = (uint8_t)(1 + below(70));
        hc_codebook cb;
        const hc_status st = hc_codebook_from_lengths(L, &cb);
        CHECK(st == HC_OK || st == HC_ERR_INVALID_ARG || st == HC_ERR_CODE_TOO_LONG);
        if (st == HC_OK && cb.max_len > 0) {
            static hc::DevTables t;
            hc::build_dev_tables(cb, &t);
        }
    }
}

void check_oracle_coding()
{
    for (int it = 0; it < 3000; ++it) {
        const uint64_t n = below(5000);
        const uint64_t B = 1 + below(600);
        std::vector<uint8_t> x(n + 1);
        const int alphabet = 1 + (int)below(256);
        for (uint64_t j = 0; j < n; ++j) x[j] = (uint8_t)below(alphabet);
        uint64_t h[256];
        or_histogram(x.data(), n, h);
        uint8_t L[256];
        uint64_t C[256];
        if (or_code_lengths(h, L) != 0) continue;
        if (n == 0) L[0] = 1;
        if (or_canonical_codes(L, C) != 0) continue;
        const uint64_t nb = (n + B - 1) / B;
        const uint64_t cap = or_encoded_size(x.data(), n, B, L);
        std::vector<uint8_t> s(cap + 1);
        std::vector<uint64_t> off(nb + 1), bits(nb + 1);
        CHECK(or_encode(x.data(), n, B, L, C, s.data(), cap, off.data(), bits.data()) == 0);
        std::vector<uint8_t> y(n + 1);
        CHECK(or_decode(s.data(), cap, n, B, L, y.data()) == 0);
        CHECK(memcmp(x.data(), y.data(), n) == 0);
        std::vector<uint64_t> w(nb + 1);
        CHECK(or_walk(s.data(), cap, nb, w.data()) == 0);
        if (cap) {  // a corrupted copy decodes or is rejected, within bounds either way
            std::vector<uint8_t> bad(s);
            bad[below(cap)] ^= (uint8_t)(1 + below(255));
            (void)or_walk(bad.data(), cap, nb, w.data());
            (void)or_decode(bad.data(), cap, n, B, L, y.data());
            (void)or_decode(bad.data(), cap - 4 * (cap >= 4), n, B, L, y.data());
        }
    }
}

void check_entry_point_arguments()
{
    for (int s = -1; s <= 9; ++s) CHECK(hc_status_str(s) != nullptr);
    CHECK(hc_encode_bound(10, 0, 8) == 0 && hc_encode_bound(10, 16, 65) == 0);
    CHECK(hc_encode_bound(~0ull >> 8, 1u << 26, 64) > 0);
    CHECK(hc_encode_workspace_bytes(10, 0) == 0);
    for (int it = 0; it < 2000; ++it) {
        const uint64_t n = next_u64() >> below(64);
        const uint32_t B = 16u * (uint32_t)(1 + below(1u << 22));
        (void)hc_encode_workspace_bytes(n >> 20, B);
        (void)hc_sub_index_entries(n >> 20, B, 16u * (uint32_t)below(64));
    }
    // a host-side handle: the checks read its host codebook, never its device tables
    uint64_t h[256];
    for (int v = 0; v < 256; ++v) h[v] = 1 + (uint64_t)v;
    hc_cb_dev_s handle;
    memset(&handle, 0, sizeof(handle));
    CHECK(hc_build_codebook(h, &handle.host) == HC_OK);
    hc_cb_handle cb = &handle;
    alignas(256) static uint8_t buf[1 << 16];
    uint8_t *p16 = buf, *odd = buf + 1;
    uint64_t *off = reinterpret_cast<uint64_t *>(buf + 4096);
    uint32_t *err = reinterpret_cast<uint32_t *>(buf + 8192);
    // null, misaligned, bad sizes: refused before any launch
    CHECK(hc_histogram(nullptr, 16, reinterpret_cast<uint64_t *>(p16), nullptr) == HC_ERR_INVALID_ARG);
    CHECK(hc_histogram(odd, 16, reinterpret_cast<uint64_t *>(p16), nullptr) == HC_ERR_INVALID_ARG);
    CHECK(hc_encode_blocks(p16, 100, 15, cb, p16, 1 << 12, off, nullptr, 0, p16, 1 << 12, err, nullptr) ==
          HC_ERR_INVALID_ARG);
    CHECK(hc_encode_blocks(p16, 100, 16, cb, p16, 1, off, nullptr, 0, p16, 1 << 12, err, nullptr) == HC_ERR_NO_SPACE);
    CHECK(hc_encode_blocks(odd, 100, 16, cb, p16, 1 << 12, off, nullptr, 0, p16, 1 << 12, err, nullptr) ==
          HC_ERR_INVALID_ARG);
    CHECK(hc_encode_blocks(p16, 100, 16, nullptr, p16, 1 << 12, off, nullptr, 0, p16, 1 << 12, err, nullptr) ==
          HC_ERR_INVALID_ARG);
    CHECK(hc_encode_blocks(p16, 100, 16, cb, p16, 1 << 12, off, nullptr, 16, p16, 1 << 12, err, nullptr) ==
          HC_ERR_INVALID_ARG);
    CHECK(hc_decode_blocks(p16, 64, 100, 16, cb, nullptr, nullptr, 0, p16, err, nullptr) == HC_ERR_INVALID_ARG);
    CHECK(hc_decode_blocks(p16, 66, 100, 16, cb, off, nullptr, 0, p16, err, nullptr) == HC_ERR_INVALID_ARG);
    CHECK(hc_decode_blocks_selfsync(p16, 64, 100, 8, cb, off, p16, err, nullptr) == HC_ERR_INVALID_ARG);
    CHECK(hc_walk_blocks(odd, 64, 4, off, err, nullptr) == HC_ERR_INVALID_ARG);
    // valid arguments reach the (stubbed) launches: the job-table logic runs on the host
    CHECK(hc_encode_blocks(p16, 1000, 64, cb, p16 + 4096 * 4, 1 << 14, off, nullptr, 0, p16 + 8192 * 4, 1 << 14,
                           err, nullptr) == HC_ERR_HIP);
    CHECK(hc_decode_blocks(p16, 64, 1000, 64, cb, off, nullptr, 0, p16, err, nullptr) == HC_ERR_HIP);
    for (int it = 0; it < 500; ++it) {
        const uint32_t count = 1 + (uint32_t)below(64);
        std::vector<hc_item> items(count);
        for (uint32_t k = 0; k < count; ++k) {
            hc_item &t = items[k];
            memset(&t, 0, sizeof(t));
            t.in = below(8) ? p16 : odd;
            t.n = below(100000);
            t.in_bytes = 4 * below(1000);
            t.cb = below(8) ? cb : nullptr;
            t.out = p16;
            t.out_cap = below(1 << 20);
            t.block_off = off;
            t.sub_idx = nullptr;
            t.hist = reinterpret_cast<uint64_t *>(p16);
        }
        const uint32_t B = 16u * (uint32_t)(1 + below(4096));
        const uint64_t need = hc_batch_workspace_bytes(items.data(), count, B);
        const uint64_t ws_bytes = below(2) ? need : below(need + 1);
        // the workspace pointer is never dereferenced on the host
        void *ws = reinterpret_cast<void *>(uintptr_t(1) << 40);
        (void)hc_histogram_batch(items.data(), count, ws, ws_bytes, nullptr);
        (void)hc_encode_batch(items.data(), count, B, 0, ws, ws_bytes, err, nullptr);
        (void)hc_decode_batch(items.data(), count, B, 0, ws, ws_bytes, err, nullptr);
    }
}

}  // namespace

int main()
{
    check_codebooks();
    check_oracle_coding();
    check_entry_point_arguments();
    if (g_fail) return 1;
    printf("host checks OK\n");
    return 0;
}
