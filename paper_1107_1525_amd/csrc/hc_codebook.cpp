// Host-side code construction: Huffman code lengths with a two-queue merge,
// canonical code values, and the decode lookup tables (paper section 2, Fig. 2).
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "hc_internal.h"

namespace hc {

hc_status canonical_from_lengths(const uint8_t *len, hc_codebook *out)
{
    hc_codebook cb;
    memset(&cb, 0, sizeof(cb));
    std::vector<int> order;
    for (int v = 0; v < kNumSym; ++v) {
        if (len[v] > kMaxLen) return HC_ERR_CODE_TOO_LONG;
        cb.len[v] = len[v];
        if (len[v]) order.push_back(v);
    }
    if (order.empty()) {
        *out = cb;
        return HC_OK;
    }
    // Kraft: sum 2^(64-len) <= 2^64, summed in 128 bits so no term overflows.
    unsigned __int128 kraft = 0;
    for (int v : order) kraft += (unsigned __int128)1 << (kMaxLen - len[v]);
    if (kraft > ((unsigned __int128)1 << kMaxLen)) return HC_ERR_INVALID_ARG;

    // Canonical values: walk the symbols by (length, value); each code is the
    // previous one plus one, shifted left by the growth in length.
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return len[a] < len[b]; });
    uint64_t code = 0;
    int prev = len[order[0]];
    for (size_t k = 0; k < order.size(); ++k) {
        int v = order[k];
        if (k > 0) code = (code + 1) << (len[v] - prev);
        prev = len[v];
        cb.code[v] = code;
        cb.max_len = std::max<uint32_t>(cb.max_len, len[v]);
    }
    cb.nsym = (uint32_t)order.size();
    *out = cb;
    return HC_OK;
}

void build_dev_tables(const hc_codebook &cb, DevTables *t)
{
    memset(t, 0, sizeof(*t));
    t->max_len = cb.max_len;
    t->nsym = cb.nsym;
    t->lut_bits = cb.max_len == 0 ? 1 : std::min<uint32_t>(cb.max_len, kLutBits);
    const uint32_t K = t->lut_bits;
    t->fixed_len = cb.max_len;
    for (int v = 0; v < kNumSym; ++v)
        if (cb.len[v] && cb.len[v] != cb.max_len) t->fixed_len = 0;

    for (int v = 0; v < kNumSym; ++v) {
        t->enc_len[v] = cb.len[v];
        t->len4[v >> 2] |= (uint32_t)cb.len[v] << (8 * (v & 3));
        t->enc_code[v] = cb.code[v];
        t->enc_packed[v] = cb.max_len <= (uint32_t)kPackedMaxLen
                               ? (uint32_t)((cb.code[v] << 8) | cb.len[v])
                               : 0u;
        if (cb.len[v]) t->count[cb.len[v]] += 1;
    }
    // symbols in canonical order (length, value): counting sort by length
    uint32_t pos = 0;
    for (int L = 1; L <= kMaxLen; ++L) {
        t->base[L] = pos;
        pos += t->count[L];
    }
    uint32_t fill[kMaxLen + 1];
    for (int L = 0; L <= kMaxLen; ++L) fill[L] = t->base[L];
    for (int v = 0; v < kNumSym; ++v) {
        const uint32_t L = cb.len[v];
        if (!L) continue;
        if (fill[L] == t->base[L]) t->first[L] = cb.code[v];  // codes of one length rise with the value
        t->sorted[fill[L]++] = (uint32_t)v;
    }
    for (uint32_t e = 0; e < (1u << K); ++e) t->lut[e] = kLutInvalid;
    for (int v = 0; v < kNumSym; ++v) {
        const uint32_t L = cb.len[v];
        if (L == 0) continue;
        if (L <= K) {
            const uint32_t lo = (uint32_t)(cb.code[v] << (K - L));
            const uint32_t hi = (uint32_t)((cb.code[v] + 1) << (K - L));
            for (uint32_t e = lo; e < hi; ++e) t->lut[e] = (uint16_t)(((uint32_t)v << 8) | L);
        } else {
            t->lut[cb.code[v] >> (L - K)] = kLutLong;
        }
    }
}

}  // namespace hc

using namespace hc;

extern "C" hc_status hc_build_codebook(const uint64_t *h_hist, hc_codebook *out)
{
    if (!h_hist || !out) return HC_ERR_INVALID_ARG;

    struct Leaf {
        uint64_t w;
        int v;
    };
    std::vector<Leaf> leaves;
    uint64_t total = 0;
    for (int v = 0; v < kNumSym; ++v) {
        if (!h_hist[v]) continue;
        if (total + h_hist[v] < total) return HC_ERR_INVALID_ARG;
        total += h_hist[v];
        leaves.push_back({h_hist[v], v});
    }
    uint8_t len[kNumSym];
    memset(len, 0, sizeof(len));
    const int m = (int)leaves.size();
    if (m == 1) len[leaves[0].v] = 1;
    if (m >= 2) {
        // Queue 1: leaves by (weight, value).  Queue 2: merged nodes in creation
        // order, whose weights never decrease.  A leaf wins a weight tie, which is
        // the (weight, key) order with leaf keys below every merged key.
        std::stable_sort(leaves.begin(), leaves.end(),
                         [](const Leaf &a, const Leaf &b) { return a.w < b.w; });
        std::vector<uint64_t> merged_w(m - 1);
        std::vector<int> parent(2 * m - 1, -1);  // ids: leaves 0..m-1, merged m..2m-2
        int next_leaf = 0, next_merged = 0;
        auto weight = [&](int id) { return id < m ? leaves[id].w : merged_w[id - m]; };
        int created = 0;
        for (int t = 0; t < m - 1; ++t) {
            int pick[2];
            for (int k = 0; k < 2; ++k) {
                const bool have_leaf = next_leaf < m;
                const bool have_merged = next_merged < created;
                if (have_leaf && (!have_merged || leaves[next_leaf].w <= merged_w[next_merged]))
                    pick[k] = next_leaf++;
                else
                    pick[k] = m + next_merged++;
            }
            merged_w[t] = weight(pick[0]) + weight(pick[1]);
            parent[pick[0]] = parent[pick[1]] = m + t;
            created = t + 1;
        }
        // Depths from the root (the last merged node) downwards: every parent was
        // created after its children, so one descending sweep suffices.
        std::vector<int> depth(2 * m - 1, 0);
        for (int id = 2 * m - 3; id >= 0; --id) depth[id] = depth[parent[id]] + 1;
        for (int k = 0; k < m; ++k) {
            if (depth[k] > kMaxLen) return HC_ERR_CODE_TOO_LONG;
            len[leaves[k].v] = (uint8_t)depth[k];
        }
    }
    return canonical_from_lengths(len, out);
}

extern "C" hc_status hc_codebook_from_lengths(const uint8_t *h_len, hc_codebook *out)
{
    if (!h_len || !out) return HC_ERR_INVALID_ARG;
    return canonical_from_lengths(h_len, out);
}
