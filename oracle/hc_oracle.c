/*
 * hc_oracle.c -- plain, slow, obviously correct CPU oracle for block-decomposed
 * Huffman coding (Cloud, Curry, Ward, Skjellum, Bangalore: "Accelerating Lossless
 * Data Compression with GPUs").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the test suite, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code, header, table or constant with the HIP
 * library: every quantity here is recomputed from its definition.
 *
 * Every routine is written for readability, not speed: the histogram is one
 * loop, the Huffman tree uses a binary heap with an explicit tie-break, codes
 * are assigned by the canonical rule, the encoder writes one bit at a time and
 * the decoder reads one bit at a time.
 *
 * Readings of the paper that this file fixes (the paper is silent or its
 * figures are missing):
 *   - the 4-byte block header holds the number of payload bits of the block
 *     (the sum of the code lengths of its symbols, section 2.1);
 *   - the header is a little-endian u32;
 *   - payload bits fill 32-bit little-endian words most-significant bit first;
 *   - pad bits up to the next 4-byte boundary are zero;
 *   - blocks follow each other with no gap;
 *   - ties in the Huffman merge order are broken by a key: leaf v has key v,
 *     the t-th merged node has key 256 + t, and the two nodes with the smallest
 *     (weight, key) are merged first;
 *   - one distinct symbol gets a 1-bit code (0);
 *   - codes are canonical (same lengths as the Huffman tree, bits assigned in
 *     order of (length, symbol value));
 *   - the last block holds n - i*B symbols.
 *
 * Parity pins: every function is checked by the CPU test suite against closed
 * forms, invariants and brute force (Kraft equality, optimal cost, exhaustive
 * enumeration of tiny inputs, round trips, corruption rejection).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Status values of the oracle.  The numbers are chosen to equal the ones the
 * public interface documents so that tests can compare them directly. */
enum {
    OR_OK = 0,
    OR_ERR_INVALID_ARG = 1,
    OR_ERR_NO_SPACE = 2,
    OR_ERR_SYMBOL_ABSENT = 4,
    OR_ERR_BLOCK_OVERFLOW = 5,
    OR_ERR_CORRUPT = 6,
    OR_ERR_CODE_TOO_LONG = 7
};

#define OR_NSYM 256
#define OR_MAXLEN 64

/* ------------------------------------------------------------------------- */
/* Step 1 (section 2): count the appearances of every distinct symbol.       */
/* ------------------------------------------------------------------------- */
void or_histogram(const uint8_t *x, uint64_t n, uint64_t hist[OR_NSYM])
{
    for (int v = 0; v < OR_NSYM; ++v) hist[v] = 0;
    for (uint64_t j = 0; j < n; ++j) hist[x[j]] += 1;
}

/* ------------------------------------------------------------------------- */
/* Step 2 (section 2, Fig. 2): Huffman tree, code length = depth of the leaf. */
/* The two lightest nodes are merged repeatedly; the order among equal       */
/* weights is fixed by the key described in the file header.                */
/* ------------------------------------------------------------------------- */
typedef struct {
    uint64_t w;   /* weight */
    uint32_t key; /* tie-break key: leaf value, or 256 + merge index */
    uint32_t id;  /* node id: 0..255 leaves, 256.. merged nodes */
} or_node;

static int or_node_less(const or_node *a, const or_node *b)
{
    if (a->w != b->w) return a->w < b->w;
    return a->key < b->key;
}

static void or_heap_push(or_node *heap, int *size, or_node nd)
{
    int i = (*size)++;
    heap[i] = nd;
    while (i > 0) {
        int parent = (i - 1) / 2;
        if (!or_node_less(&heap[i], &heap[parent])) break;
        or_node tmp = heap[i];
        heap[i] = heap[parent];
        heap[parent] = tmp;
        i = parent;
    }
}

static or_node or_heap_pop(or_node *heap, int *size)
{
    or_node top = heap[0];
    heap[0] = heap[--(*size)];
    int i = 0;
    for (;;) {
        int l = 2 * i + 1, r = 2 * i + 2, m = i;
        if (l < *size && or_node_less(&heap[l], &heap[m])) m = l;
        if (r < *size && or_node_less(&heap[r], &heap[m])) m = r;
        if (m == i) break;
        or_node tmp = heap[i];
        heap[i] = heap[m];
        heap[m] = tmp;
        i = m;
    }
    return top;
}

/* Returns OR_OK, OR_ERR_INVALID_ARG if the weights overflow 64 bits, or
 * OR_ERR_CODE_TOO_LONG if some depth exceeds 64.  len[v] = 0 for absent v. */
int or_code_lengths(const uint64_t hist[OR_NSYM], uint8_t len[OR_NSYM])
{
    or_node heap[OR_NSYM];
    int parent[2 * OR_NSYM]; /* parent id of each node, -1 for the root */
    int size = 0, m = 0;
    uint64_t total = 0;

    for (int v = 0; v < OR_NSYM; ++v) len[v] = 0;
    for (int i = 0; i < 2 * OR_NSYM; ++i) parent[i] = -1;

    for (int v = 0; v < OR_NSYM; ++v) {
        if (hist[v] == 0) continue;
        if (total + hist[v] < total) return OR_ERR_INVALID_ARG;
        total += hist[v];
        or_node leaf = {hist[v], (uint32_t)v, (uint32_t)v};
        or_heap_push(heap, &size, leaf);
        ++m;
    }
    if (m == 0) return OR_OK;
    if (m == 1) { /* a lone symbol still needs one bit per occurrence */
        len[heap[0].id] = 1;
        return OR_OK;
    }
    for (int t = 0; t < m - 1; ++t) {
        or_node a = or_heap_pop(heap, &size);
        or_node b = or_heap_pop(heap, &size);
        or_node merged = {a.w + b.w, (uint32_t)(OR_NSYM + t), (uint32_t)(OR_NSYM + t)};
        parent[a.id] = (int)merged.id;
        parent[b.id] = (int)merged.id;
        or_heap_push(heap, &size, merged);
    }
    for (int v = 0; v < OR_NSYM; ++v) {
        if (hist[v] == 0) continue;
        int depth = 0;
        for (int node = v; parent[node] != -1; node = parent[node]) ++depth;
        if (depth > OR_MAXLEN) return OR_ERR_CODE_TOO_LONG;
        len[v] = (uint8_t)depth;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Canonical code assignment (the rule published in RFC 1951, section        */
/* 3.2.2): count codes per length, compute the first code of every length,   */
/* then hand out consecutive codes in increasing symbol order.               */
/* ------------------------------------------------------------------------- */
int or_canonical_codes(const uint8_t len[OR_NSYM], uint64_t code[OR_NSYM])
{
    uint64_t bl_count[OR_MAXLEN + 1];
    uint64_t next_code[OR_MAXLEN + 2];
    int max_len = 0;

    for (int L = 0; L <= OR_MAXLEN; ++L) bl_count[L] = 0;
    for (int v = 0; v < OR_NSYM; ++v) {
        code[v] = 0;
        if (len[v] > OR_MAXLEN) return OR_ERR_CODE_TOO_LONG;
        if (len[v] > 0) {
            bl_count[len[v]] += 1;
            if (len[v] > max_len) max_len = len[v];
        }
    }
    uint64_t c = 0;
    next_code[0] = 0;
    for (int L = 1; L <= max_len; ++L) {
        c = (c + (L >= 2 ? bl_count[L - 1] : 0)) << 1;
        next_code[L] = c;
    }
    for (int v = 0; v < OR_NSYM; ++v) {
        if (len[v] == 0) continue;
        code[v] = next_code[len[v]];
        next_code[len[v]] += 1;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Block layout (section 2.1, Fig. 3 and 4).                                  */
/* ------------------------------------------------------------------------- */
uint64_t or_num_blocks(uint64_t n, uint64_t B)
{
    if (B == 0) return 0;
    return (n + B - 1) / B;
}

/* Bytes a block occupies: the 4-byte header plus the payload rounded up to a
 * whole number of 4-byte words. */
uint64_t or_block_bytes(uint64_t bits)
{
    return 4 + 4 * ((bits + 31) / 32);
}

/* Writes one bit at payload bit position p of a block whose payload starts at
 * byte 'base' of 'out' (words are little-endian, filled from bit 31 down). */
static void or_put_bit(uint8_t *out, uint64_t base, uint64_t p, int bit)
{
    if (!bit) return;
    uint64_t word = p / 32;
    int pos_in_word = 31 - (int)(p % 32); /* bit number within the u32 */
    uint64_t byte = base + 4 * word + (uint64_t)(pos_in_word / 8);
    out[byte] |= (uint8_t)(1u << (pos_in_word % 8));
}

static int or_get_bit(const uint8_t *in, uint64_t base, uint64_t p)
{
    uint64_t word = p / 32;
    int pos_in_word = 31 - (int)(p % 32);
    uint64_t byte = base + 4 * word + (uint64_t)(pos_in_word / 8);
    return (in[byte] >> (pos_in_word % 8)) & 1;
}

static void or_put_u32le(uint8_t *out, uint64_t at, uint32_t v)
{
    out[at + 0] = (uint8_t)(v);
    out[at + 1] = (uint8_t)(v >> 8);
    out[at + 2] = (uint8_t)(v >> 16);
    out[at + 3] = (uint8_t)(v >> 24);
}

static uint32_t or_get_u32le(const uint8_t *in, uint64_t at)
{
    return (uint32_t)in[at] | ((uint32_t)in[at + 1] << 8) | ((uint32_t)in[at + 2] << 16) |
           ((uint32_t)in[at + 3] << 24);
}

/* Length pass (section 2.1): bits[i] = sum of the code lengths of the symbols
 * of block i.  Fails with SYMBOL_ABSENT on a symbol without a code and with
 * BLOCK_OVERFLOW if a sum does not fit the 4-byte header. */
int or_block_bits(const uint8_t *x, uint64_t n, uint64_t B, const uint8_t len[OR_NSYM],
                  uint64_t *bits /* nb entries */)
{
    if (B == 0) return OR_ERR_INVALID_ARG;
    uint64_t nb = or_num_blocks(n, B);
    for (uint64_t i = 0; i < nb; ++i) {
        uint64_t first = i * B;
        uint64_t last = first + B < n ? first + B : n;
        uint64_t sum = 0;
        for (uint64_t j = first; j < last; ++j) {
            if (len[x[j]] == 0) return OR_ERR_SYMBOL_ABSENT;
            sum += len[x[j]];
        }
        if (sum > 0xFFFFFFFFull) return OR_ERR_BLOCK_OVERFLOW;
        bits[i] = sum;
    }
    return OR_OK;
}

/* Total encoded size C (bytes) of x under the given lengths, or 0 on error. */
uint64_t or_encoded_size(const uint8_t *x, uint64_t n, uint64_t B, const uint8_t len[OR_NSYM])
{
    uint64_t nb = or_num_blocks(n, B), total = 0;
    uint64_t *bits = (uint64_t *)malloc((nb ? nb : 1) * sizeof(uint64_t));
    if (!bits) return 0;
    if (or_block_bits(x, n, B, len, bits) != OR_OK) {
        free(bits);
        return 0;
    }
    for (uint64_t i = 0; i < nb; ++i) total += or_block_bytes(bits[i]);
    free(bits);
    return total;
}

/* Encoder (section 2.1, Fig. 3 and 4).  For every block: the header (payload
 * bit count), then every symbol's code emitted bit by bit from its most
 * significant bit, then zero pad to a 4-byte boundary.  Blocks are written back
 * to back; offsets[i] is the byte position of block i's header and
 * offsets[nb] = C.  'bits' (nb entries) receives the header values. */
int or_encode(const uint8_t *x, uint64_t n, uint64_t B, const uint8_t len[OR_NSYM],
              const uint64_t code[OR_NSYM], uint8_t *out, uint64_t out_cap,
              uint64_t *offsets /* nb + 1 */, uint64_t *bits /* nb */)
{
    if (B == 0) return OR_ERR_INVALID_ARG;
    uint64_t nb = or_num_blocks(n, B);
    int st = or_block_bits(x, n, B, len, bits);
    if (st != OR_OK) return st;

    offsets[0] = 0;
    for (uint64_t i = 0; i < nb; ++i) offsets[i + 1] = offsets[i] + or_block_bytes(bits[i]);
    if (offsets[nb] > out_cap) return OR_ERR_NO_SPACE;
    memset(out, 0, offsets[nb]);

    for (uint64_t i = 0; i < nb; ++i) {
        or_put_u32le(out, offsets[i], (uint32_t)bits[i]);
        uint64_t payload = offsets[i] + 4;
        uint64_t p = 0;
        uint64_t first = i * B;
        uint64_t last = first + B < n ? first + B : n;
        for (uint64_t j = first; j < last; ++j) {
            int L = len[x[j]];
            for (int b = L - 1; b >= 0; --b) {
                or_put_bit(out, payload, p, (int)((code[x[j]] >> b) & 1u));
                p += 1;
            }
        }
        /* p == bits[i] by construction; the pad bits stay zero. */
    }
    return OR_OK;
}

/* Sub-block index (an extension of the offset table of section 2.1): for block
 * i and chunk c (chunks of S symbols), idx[i * cpb + c] is the payload bit
 * position of symbol c*S of the block, or the block's bit count if the block
 * has no such symbol; cpb = ceil(B / S). */
int or_sub_index(const uint8_t *x, uint64_t n, uint64_t B, uint64_t S, const uint8_t len[OR_NSYM],
                 uint32_t *idx)
{
    if (B == 0 || S == 0) return OR_ERR_INVALID_ARG;
    uint64_t nb = or_num_blocks(n, B);
    uint64_t cpb = (B + S - 1) / S;
    for (uint64_t i = 0; i < nb; ++i) {
        uint64_t first = i * B;
        uint64_t cnt = (first + B < n ? first + B : n) - first;
        uint64_t p = 0;
        for (uint64_t k = 0; k < cnt; ++k) {
            if (k % S == 0) idx[i * cpb + k / S] = (uint32_t)p;
            p += len[x[first + k]];
        }
        for (uint64_t c = 0; c < cpb; ++c)
            if (c * S >= cnt) idx[i * cpb + c] = (uint32_t)p;
    }
    return OR_OK;
}

/* Header walk (section 2.1): the offset table rebuilt from the length
 * delimiters alone.  Checks every block lies inside the stream and that the
 * last block ends exactly at in_bytes. */
int or_walk(const uint8_t *in, uint64_t in_bytes, uint64_t nb, uint64_t *offsets /* nb + 1 */)
{
    offsets[0] = 0;
    for (uint64_t i = 0; i < nb; ++i) {
        if (offsets[i] + 4 > in_bytes) return OR_ERR_CORRUPT;
        uint64_t bits = or_get_u32le(in, offsets[i]);
        offsets[i + 1] = offsets[i] + or_block_bytes(bits);
        if (offsets[i + 1] > in_bytes) return OR_ERR_CORRUPT;
    }
    if (offsets[nb] != in_bytes) return OR_ERR_CORRUPT;
    return OR_OK;
}

/* Strict decoder (section 2.1 and 3.2).  Each block's symbols are read one
 * bit at a time: the bits read so far form a value c of length L, and a code
 * is recognised when c falls inside the range of canonical codes of length L.
 * The block must use exactly its header's bit count, its pad bits must be
 * zero, and the blocks must tile the stream exactly. */
int or_decode(const uint8_t *in, uint64_t in_bytes, uint64_t n, uint64_t B,
              const uint8_t len[OR_NSYM], uint8_t *out)
{
    if (B == 0) return OR_ERR_INVALID_ARG;
    uint64_t count[OR_MAXLEN + 1];
    uint64_t first[OR_MAXLEN + 1];
    uint64_t base[OR_MAXLEN + 1];
    uint8_t sorted[OR_NSYM];
    int max_len = 0, nsorted = 0;

    for (int L = 0; L <= OR_MAXLEN; ++L) count[L] = first[L] = base[L] = 0;
    for (int v = 0; v < OR_NSYM; ++v) {
        if (len[v] > OR_MAXLEN) return OR_ERR_CODE_TOO_LONG;
        if (len[v] > 0) {
            count[len[v]] += 1;
            if (len[v] > max_len) max_len = len[v];
        }
    }
    /* symbols sorted by (length, value): the canonical order */
    for (int L = 1; L <= max_len; ++L) {
        base[L] = (uint64_t)nsorted;
        for (int v = 0; v < OR_NSYM; ++v)
            if (len[v] == L) sorted[nsorted++] = (uint8_t)v;
    }
    uint64_t c = 0;
    for (int L = 1; L <= max_len; ++L) {
        c = (c + (L >= 2 ? count[L - 1] : 0)) << 1;
        first[L] = c;
    }

    uint64_t nb = or_num_blocks(n, B);
    uint64_t off = 0;
    for (uint64_t i = 0; i < nb; ++i) {
        if (off + 4 > in_bytes) return OR_ERR_CORRUPT;
        uint64_t bits = or_get_u32le(in, off);
        uint64_t bytes = or_block_bytes(bits);
        if (off + bytes > in_bytes) return OR_ERR_CORRUPT;
        uint64_t payload = off + 4;
        uint64_t first_sym = i * B;
        uint64_t cnt = (first_sym + B < n ? first_sym + B : n) - first_sym;
        uint64_t p = 0;
        for (uint64_t k = 0; k < cnt; ++k) {
            uint64_t value = 0;
            int L = 0;
            for (;;) {
                if (p >= bits) return OR_ERR_CORRUPT; /* code runs past the header's count */
                value = (value << 1) | (uint64_t)or_get_bit(in, payload, p);
                p += 1;
                L += 1;
                if (L > max_len) return OR_ERR_CORRUPT;
                if (value >= first[L] && value - first[L] < count[L]) break;
            }
            out[first_sym + k] = sorted[base[L] + (value - first[L])];
        }
        if (p != bits) return OR_ERR_CORRUPT; /* unused payload bits */
        for (uint64_t q = bits; q < 32 * ((bits + 31) / 32); ++q)
            if (or_get_bit(in, payload, q)) return OR_ERR_CORRUPT; /* nonzero pad */
        off += bytes;
    }
    if (off != in_bytes) return OR_ERR_CORRUPT; /* trailing bytes */
    return OR_OK;
}
