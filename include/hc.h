/*
 * hc.h -- C ABI of the MI355X (gfx950) block-decomposed Huffman codec.
 *
 * The method is the one of Cloud, Curry, Ward, Skjellum and Bangalore,
 * "Accelerating Lossless Data Compression with GPUs": the symbols of the input
 * are counted (section 2), a Huffman code is built from the counts (section 2,
 * Fig. 2), the input is cut into blocks holding a constant number of symbols
 * which are encoded independently, each block carrying a 4-byte length
 * delimiter and padded to a 4-byte boundary (section 2.1, Fig. 3 and 4), and
 * decoding runs in parallel over the blocks from a table of block offsets
 * (section 2.1, section 3.2).
 *
 * Stream format (one "stream" = the encoding of one input buffer):
 *   for every block i = 0 .. nb-1, back to back, with no gap:
 *     u32 little-endian  bits_i   number of payload bits of block i
 *                                 (the sum of the code lengths of its symbols)
 *     ceil(bits_i/32) little-endian u32 payload words; the code words of the
 *                                 block's symbols fill them from bit 31 down to
 *                                 bit 0, word after word; unused bits are 0.
 *   Block i holds symbols [i*B, min(n, (i+1)*B)) of the input, nb = ceil(n/B).
 *   Block offsets: off[0] = 0, off[i+1] = off[i] + 4 + 4*ceil(bits_i/32),
 *   C = off[nb] is the stream size in bytes.
 *   Codes are canonical Huffman codes (lengths from the Huffman tree, values
 *   assigned in order of (length, symbol)), up to 64 bits long.
 *
 * Conventions shared by all entry points:
 *   - Pointers named d_* are device memory owned by the caller; h_* are host
 *     memory owned by the caller.  The library allocates memory only in
 *     hc_codebook_upload and hc_cbset_create (freed by hc_codebook_destroy and
 *     hc_cbset_destroy), the pinned staging ring of the batch calls' job
 *     tables (see hc_histogram_batch: on first use and when a table outgrows
 *     it), and, once per device, the batch calls' side streams and events
 *     (see hc_decode_batch), all kept until the process ends; no other call
 *     allocates or frees.  Calls that wait on the host: hc_codebook_upload
 *     (its copy), hc_codebook_update and hc_cbset_build (the handle's or
 *     set's own previous table copy, normally long finished),
 *     hc_codebook_destroy and hc_cbset_destroy (the same, and the runtime's
 *     free), and a batch call whose staging buffer (used again every eighth
 *     call) still holds a copy that has not left it (normally long
 *     finished).  The other coding calls never wait.
 *   - 'stream' is a hipStream_t passed as void* (NULL = the null stream).
 *     Device work is enqueued on it and the call returns without waiting.
 *   - Errors that the host can see (bad sizes, null or misaligned pointers,
 *     too small buffers) are returned at once and enqueue nothing.
 *   - Errors that only the data reveals (a symbol without a code, a block
 *     longer than 2^32-1 bits, a corrupt stream) are written by the kernels to
 *     the caller's u32 error word d_err: a kernel writes its code only if the
 *     word still holds 0, so the word keeps the first error.  Zero it before a
 *     sequence of calls and read it after synchronising.  After any error the
 *     outputs of the failing call are unspecified.
 *   - Results depend only on the inputs (bytes, n, B, S and the codebook),
 *     never on launch shape or on the order in which atomics land.
 *   - No call aborts, exits or throws.  Calls on different streams may run
 *     concurrently as long as they write to different buffers.
 *   - Alignment: d_in of hc_histogram / hc_encode_blocks / hc_decode_blocks
 *     and d_out of hc_encode_blocks / hc_decode_blocks must be 16-byte
 *     aligned; the stream of hc_walk_blocks 4-byte aligned; u64 arrays
 *     8-byte aligned.
 *   - Limits: 16 <= B <= 2^26 and B % 16 == 0; sub-block stride S is 0 (no
 *     sub-block index) or a multiple of 16.
 */
#ifndef HC_H
#define HC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HC_OK = 0,
    HC_ERR_INVALID_ARG = 1,    /* bad size, null or misaligned pointer, bad codebook */
    HC_ERR_NO_SPACE = 2,       /* an output or workspace buffer is too small */
    HC_ERR_HIP = 3,            /* the HIP runtime reported an error */
    HC_ERR_SYMBOL_ABSENT = 4,  /* the input holds a symbol the codebook has no code for */
    HC_ERR_BLOCK_OVERFLOW = 5, /* a block's bit count does not fit the 4-byte header */
    HC_ERR_CORRUPT = 6,        /* the compressed stream is not a valid encoding */
    HC_ERR_CODE_TOO_LONG = 7,  /* a Huffman code would be longer than 64 bits */
    HC_ERR_TABLE_CHANGED = 8   /* (in d_err) a launch met code tables other than those it
                                  was shaped for: a replayed graph whose codes got longer
                                  or stopped being complete 8-bit codes */
} hc_status;

/* Host description of a code: lengths and canonical code values.
 * len[v] = 0 means symbol v has no code; code[v] holds len[v] bits,
 * right-aligned (the first bit of the code word is bit len[v]-1). */
typedef struct {
    uint8_t len[256];
    uint64_t code[256];
    uint32_t max_len; /* longest code length, 0 if no symbol has a code */
    uint32_t nsym;    /* number of symbols with a code */
} hc_codebook;

/* Device-resident copy of a codebook with its encode table and decode lookup
 * tables.  Owned by the library. */
typedef struct hc_cb_dev_s *hc_cb_handle;

/* Human-readable name of a status value (static storage, never NULL). */
const char *hc_status_str(int status);

/* Library version: major * 10000 + minor * 100 + patch. */
int hc_version(void);

/* Launch parameters an autotuner may set for the whole process (a         */
/* measurement helper, not part of the method): they change how the       */
/* kernels cut the work, never a byte of any output.                       */
typedef struct {
    uint32_t encode_tile_loads; /* 16-byte loads per thread of an encode tile (a tile is
                                   4096 times as many symbols): 0 = the library's rule
                                   (4 for blocks of >= 16 Ki symbols and codes of <= 16
                                   bits, 2 for blocks of >= 8 Ki, else 1); 1, 2 or 4 caps it */
} hc_tuning;

/* Sets the parameters for launches made after the call (a captured graph  */
/* keeps the ones it was captured with).  Errors: INVALID_ARG (null, or    */
/* encode_tile_loads not 0, 1, 2 or 4).                                    */
hc_status hc_set_tuning(const hc_tuning *t);
/* Reads the current parameters.  Errors: INVALID_ARG (null).              */
hc_status hc_get_tuning(hc_tuning *t);

/* ---------------------------------------------------------------------- */
/* Symbol statistics (section 2: count every distinct symbol).            */
/* d_hist[v] = number of bytes equal to v among d_in[0 .. n-1].           */
/* d_in: n bytes, 16-byte aligned (may be NULL if n == 0).                */
/* d_hist: 256 u64, overwritten (zeroed first, then filled).              */
/* Errors: INVALID_ARG (null/misaligned pointer), HIP.                    */
/* ---------------------------------------------------------------------- */
hc_status hc_histogram(const uint8_t *d_in, uint64_t n, uint64_t *d_hist, void *stream);

/* ---------------------------------------------------------------------- */
/* Code construction (section 2, Fig. 2), on the host.                    */
/* Huffman code lengths from the 256 counts h_hist, then canonical code   */
/* values.  Ties among equal weights are broken by a key (leaf v has key  */
/* v, the t-th merged node key 256+t; the two smallest (weight, key) are  */
/* merged first), so equal counts always give the same code.  A single    */
/* present symbol gets a 1-bit code; no present symbol gives an empty     */
/* codebook (max_len = 0).                                                */
/* Errors: INVALID_ARG (null pointer, counts summing past 2^64-1),        */
/* CODE_TOO_LONG (a code would exceed 64 bits).                           */
/* ---------------------------------------------------------------------- */
hc_status hc_build_codebook(const uint64_t *h_hist, hc_codebook *out);

/* Canonical codebook for given code lengths (for codes built elsewhere).  */
/* The lengths must satisfy Kraft's inequality (sum 2^-len <= 1).         */
/* Errors: INVALID_ARG (null pointer, Kraft sum above 1),                 */
/* CODE_TOO_LONG (a length above 64).                                     */
hc_status hc_codebook_from_lengths(const uint8_t *h_len, hc_codebook *out);

/* Copies a codebook and its lookup tables to the current device.  The    */
/* handle stays valid until hc_codebook_destroy.  Synchronous (allocates  */
/* device memory, a pinned host staging area and an event, and copies     */
/* with hipMemcpy).                                                       */
/* Errors: INVALID_ARG (null pointer, inconsistent codebook), HIP.        */
hc_status hc_codebook_upload(const hc_codebook *cb, hc_cb_handle *out);

/* Replaces the tables of an existing handle with those of another        */
/* codebook without allocating: the tables are built on the host into a   */
/* pinned staging area owned by the handle and copied asynchronously on   */
/* 'stream'.  Work enqueued earlier on that stream still sees the old     */
/* tables, work enqueued later the new ones; work on other streams that   */
/* reads the handle must be ordered by the caller.  Waits (host side) for */
/* the handle's previous update copy to finish before reusing the         */
/* staging area.                                                          */
/* Errors: INVALID_ARG (null pointer, inconsistent codebook), HIP.        */
hc_status hc_codebook_update(hc_cb_handle h, const hc_codebook *cb, void *stream);

/* A codebook set: 'count' device-resident code tables in one allocation, */
/* rebuilt together from 'count' histograms with one asynchronous copy.   */
/* For streams that get a new code every step (one per segment or        */
/* buffer).  Owned by the library; the handles from hc_cbset_handle are   */
/* valid until hc_cbset_destroy and must not be passed to                 */
/* hc_codebook_update or hc_codebook_destroy (which ignores them).         */
typedef struct hc_cbset_s *hc_cbset;

/* Allocates a set of 'count' tables (device memory, pinned staging, an   */
/* event); every table starts as the empty code.  Synchronous.            */
/* Errors: INVALID_ARG (count 0, null pointer), HIP.                       */
hc_status hc_cbset_create(uint32_t count, hc_cbset *out);

/* Handle of table k of the set (NULL if k is out of range).              */
hc_cb_handle hc_cbset_handle(hc_cbset set, uint32_t k);

/* Builds code k from histogram k (h_hists: count x 256 u64, host) for     */
/* every k, exactly as hc_build_codebook (an all-zero histogram gets the  */
/* one-symbol code {0: 1 bit}), writes the codebooks to h_out (count, may */
/* be NULL), and refreshes the device tables with one asynchronous copy   */
/* on 'stream': work enqueued later on that stream sees the new tables.   */
/* Waits (host side) for the set's previous copy before reusing the       */
/* staging area.  The codes are built on up to eight host threads, the    */
/* calling one included.  Errors: INVALID_ARG, CODE_TOO_LONG, HIP.         */
hc_status hc_cbset_build(hc_cbset set, const uint64_t *h_hists, hc_codebook *h_out, void *stream);

/* Frees a set (NULL is accepted).  Waits for the set's own last table    */
/* copy, not for the device; the caller must have ordered every launch     */
/* that reads the set's tables before the call (a stream or event          */
/* synchronisation), as for any freed buffer.                              */
hc_status hc_cbset_destroy(hc_cbset set);

/* Frees a handle from hc_codebook_upload (NULL is accepted).  Waits for  */
/* the handle's own last table copy only; launches that read the handle   */
/* must be finished (ordered by the caller) before the call.              */
hc_status hc_codebook_destroy(hc_cb_handle cb);

/* ---------------------------------------------------------------------- */
/* Block encoding (section 2.1, Fig. 3 and 4).                            */
/* ---------------------------------------------------------------------- */

/* Upper bound of the stream size C for n symbols, block size B and codes */
/* of at most max_len bits: sum over blocks of 4 + 4*ceil(cnt*max_len/32). */
/* Returns 0 for B == 0 or max_len > 64.                                  */
uint64_t hc_encode_bound(uint64_t n, uint32_t block_size, uint32_t max_len);

/* Bytes of device workspace hc_encode_blocks needs for n and B.          */
uint64_t hc_encode_workspace_bytes(uint64_t n, uint32_t block_size);

/* Number of u32 entries of the sub-block index for n, B and S (0 if S == 0):
 * nb * ceil(B / S). */
uint64_t hc_sub_index_entries(uint64_t n, uint32_t block_size, uint32_t sub_block);

/* Encodes d_in[0 .. n-1] into d_out in the stream format above.
 *   block_size   B, symbols per block.
 *   cb           device codebook; every symbol of the input needs a code
 *                (else SYMBOL_ABSENT in *d_err).
 *   d_out        out_cap bytes, 16-byte aligned; out_cap must be at least
 *                hc_encode_bound(n, B, cb max_len).  Bytes past C are left
 *                untouched.
 *   d_block_off  nb + 1 u64: off[i] = byte offset of block i's header,
 *                off[nb] = C (the offset table of section 2.1, produced here
 *                by an exclusive scan of the block sizes).
 *   d_sub_idx    NULL, or hc_sub_index_entries(n, B, S) u32: for block i and
 *                chunk c, entry i*ceil(B/S)+c is the payload bit position of
 *                the block's symbol c*S (the block's bit count if the block
 *                has no such symbol).  An extension of the offset table that
 *                lets decoding split a block into chunks of S symbols.
 *   sub_block    S; must be 0 when d_sub_idx is NULL.
 *   d_ws         hc_encode_workspace_bytes(n, B) bytes of device scratch,
 *                8-byte aligned, owned by the caller; contents on entry are
 *                ignored.
 *   d_err        u32 error word (see conventions).
 * Errors returned: INVALID_ARG, NO_SPACE, HIP.  Errors in *d_err:
 * SYMBOL_ABSENT, BLOCK_OVERFLOW. */
hc_status hc_encode_blocks(const uint8_t *d_in, uint64_t n, uint32_t block_size, hc_cb_handle cb,
                           uint8_t *d_out, uint64_t out_cap, uint64_t *d_block_off,
                           uint32_t *d_sub_idx, uint32_t sub_block, void *d_ws, uint64_t ws_bytes,
                           uint32_t *d_err, void *stream);

/* Size in bytes of the device array that hc_encode_blocks_noalloc uses as  */
/* its scratch (one copy per GPU, held until the process ends).            */
#define HC_NOALLOC_SCRATCH_BYTES (32ull << 20)

/* hc_encode_blocks without a workspace argument, for callers that cannot  */
/* allocate device memory (code under stream capture, tight serving loops, */
/* harnesses that forbid allocation): the encoder's scratch is a           */
/* file-scope device array of HC_NOALLOC_SCRATCH_BYTES per GPU.  The call   */
/* itself allocates and frees nothing; the first call on a device looks up */
/* that device's copy of the array once.  Other arguments, layouts and     */
/* errors are those of hc_encode_blocks.                                   */
/* Limit: the scratch this (n, B, codebook) needs, as hc_encode_blocks      */
/* would use of its workspace (hc_encode_workspace_bytes(n, B) bounds it;   */
/* about n/32 bytes for B >= 16384, 8 bytes per block for B <= 4096), must  */
/* fit HC_NOALLOC_SCRATCH_BYTES, else NO_SPACE is returned and nothing is   */
/* enqueued.  Every call on one GPU shares that GPU's array and nothing in  */
/* it needs clearing (every entry is written before it is read), so calls  */
/* that may overlap in time on one GPU (different streams, or host threads */
/* without ordering) race on it: order them, e.g. on one stream.          */
/* Errors returned: INVALID_ARG, NO_SPACE, HIP; in *d_err: SYMBOL_ABSENT,   */
/* BLOCK_OVERFLOW.                                                          */
hc_status hc_encode_blocks_noalloc(const uint8_t *d_in, uint64_t n, uint32_t block_size, hc_cb_handle cb,
                                   uint8_t *d_out, uint64_t out_cap, uint64_t *d_block_off, uint32_t *d_sub_idx,
                                   uint32_t sub_block, uint32_t *d_err, void *stream);

/* ---------------------------------------------------------------------- */
/* Offset table from the length delimiters (section 2.1), for a stream    */
/* whose offsets were not kept.  Walks the nb headers one after another   */
/* (a dependent chain: latency-bound).  d_in: in_bytes of stream, 4-byte  */
/* aligned.  d_block_off: nb + 1 u64.  CORRUPT in *d_err if a block runs   */
/* past in_bytes or the last block does not end at in_bytes.               */
/* ---------------------------------------------------------------------- */
hc_status hc_walk_blocks(const uint8_t *d_in, uint64_t in_bytes, uint64_t nb, uint64_t *d_block_off,
                         uint32_t *d_err, void *stream);

/* ---------------------------------------------------------------------- */
/* Parallel block decoding (section 2.1, section 3.2).                    */
/*   d_in, in_bytes  the stream (16-byte aligned, in_bytes % 4 == 0).  The */
/*                   decoder reads whole 16-byte pieces, so the last one   */
/*                   may reach up to 12 bytes past in_bytes (within the    */
/*                   16-byte piece that holds the stream's last word; the  */
/*                   values read there never reach the output).            */
/*   n, block_size   symbol count and B used to encode.                    */
/*   cb              the encoding's codebook.                              */
/*   d_block_off     nb + 1 u64 offsets (from hc_encode_blocks or          */
/*                   hc_walk_blocks).  Required: a NULL table is refused   */
/*                   (INVALID_ARG) rather than walked here, because the    */
/*                   walk needs nb + 1 u64 of memory that this call does   */
/*                   not take and would not allocate; walk first with      */
/*                   hc_walk_blocks into a buffer of the caller's.         */
/*   d_sub_idx, sub_block  the sub-block index written by hc_encode_blocks */
/*                   with the same S, or NULL and 0: then each block is    */
/*                   decoded as one piece.                                 */
/*   d_out           n bytes, 16-byte aligned; block i goes to             */
/*                   d_out[i*B ...].                                       */
/* Decoding is strict: every block must use exactly its header's bit      */
/* count (and every chunk exactly the bits the index gives it), pad bits  */
/* must be zero, headers must agree with the offsets and the blocks must  */
/* end exactly at in_bytes; otherwise CORRUPT in *d_err.                   */
/* Errors returned: INVALID_ARG, HIP.                                      */
/* ---------------------------------------------------------------------- */
hc_status hc_decode_blocks(const uint8_t *d_in, uint64_t in_bytes, uint64_t n, uint32_t block_size,
                           hc_cb_handle cb, const uint64_t *d_block_off, const uint32_t *d_sub_idx,
                           uint32_t sub_block, uint8_t *d_out, uint32_t *d_err, void *stream);

/* ---------------------------------------------------------------------- */
/* Batches: many independent buffers, each with its own codebook, in one  */
/* launch per step (the blocks of all buffers are independent units of    */
/* work that many processors may code at once: abstract, section 2.1).    */
/* Every buffer follows the contract of the single-buffer call; B and S    */
/* are common to the batch.                                                */
/* ---------------------------------------------------------------------- */
typedef struct {
    const uint8_t *in;    /* histogram / encode: the n bytes (16-byte aligned); decode: the stream */
    uint64_t n;           /* symbols (uncompressed bytes) */
    uint64_t in_bytes;    /* decode: stream bytes C (multiple of 4); ignored otherwise */
    hc_cb_handle cb;      /* encode / decode: this buffer's codebook */
    uint8_t *out;         /* encode: stream buffer; decode: n output bytes (16-byte aligned) */
    uint64_t out_cap;     /* encode: bytes at out, at least hc_encode_bound(n, B, max_len) */
    uint64_t *block_off;  /* encode: nb + 1 offsets written; decode: read */
    uint32_t *sub_idx;    /* sub-block index (written by encode, read by decode) when S > 0, else NULL */
    uint64_t *hist;       /* histogram: 256 u64 written */
} hc_item;

/* Device workspace (256-byte aligned, caller-owned) any of the batch      */
/* calls needs for these items and block size: the job table (room for    */
/* one per launch: the encode and decode calls launch each code class     */
/* apart), then the encoder's per-tile (and per-thread) bit counts and    */
/* positions.                                                              */
uint64_t hc_batch_workspace_bytes(const hc_item *items, uint32_t count, uint32_t block_size);

/* hc_histogram for every item (uses in, n, hist).  The item table is       */
/* written into d_ws on 'stream' as one asynchronous copy from a small     */
/* ring of pinned host buffers the library keeps for all batch calls       */
/* (allocated on first use, grown when a table outgrows its buffer; a      */
/* buffer is reused once its copy has left it), or, while 'stream' is      */
/* being captured into a graph, by small kernels that carry the items as   */
/* arguments (a replay then needs no host buffer).  Nothing waits for the  */
/* stream; 'items' may be reused when the call returns.                    */
/* Errors returned: INVALID_ARG, NO_SPACE, HIP.                            */
hc_status hc_histogram_batch(const hc_item *items, uint32_t count, void *d_ws, uint64_t ws_bytes, void *stream);

/* hc_encode_blocks for every item (uses in, n, cb, out, out_cap,          */
/* block_off, sub_idx) with block size B and sub-block stride S.  Per code */
/* class present (complete 8-bit codes, which need no length pass; then    */
/* longest codes <= 16, <= 24 bits, longer) one launch of each step over   */
/* the tiles of all its items; the classes side by side as in             */
/* hc_decode_batch.  Each item's offsets start at 0 in its own stream.     */
/* Errors returned: INVALID_ARG, NO_SPACE, HIP; in *d_err: SYMBOL_ABSENT,   */
/* BLOCK_OVERFLOW, TABLE_CHANGED (graph replays: see hc_decode_batch).     */
hc_status hc_encode_batch(const hc_item *items, uint32_t count, uint32_t block_size, uint32_t sub_block,
                          void *d_ws, uint64_t ws_bytes, uint32_t *d_err, void *stream);

/* The three steps of hc_encode_batch as separate calls (section 2.1: the  */
/* block lengths, the table of where each block begins, then the          */
/* packing), for callers that time or schedule them one by one.  Same      */
/* arguments as hc_encode_batch; issue them in this order on one stream    */
/* with the same items and workspace (the workspace carries each tile's    */
/* bit count from the first step to the second, its in-block position     */
/* from the second to the third, and for tiles of more than 4096 symbols  */
/* the bit count of each of the tile's 256 threads from the first to the  */
/* third).  Together they equal hc_encode_batch.                           */
/*   lengths: per tile of the input, the sum of its code lengths (items    */
/*            with a complete 8-bit code are left out: the offsets step    */
/*            counts 8 bits a symbol for them); in *d_err: SYMBOL_ABSENT.  */
/*   offsets: block_off of every item (C = block_off[nb]);                  */
/*            in *d_err: BLOCK_OVERFLOW.                                   */
/*   pack:    the stream (headers, code words, zero pad) and sub_idx.      */
hc_status hc_encode_lengths_batch(const hc_item *items, uint32_t count, uint32_t block_size, uint32_t sub_block,
                                  void *d_ws, uint64_t ws_bytes, uint32_t *d_err, void *stream);
hc_status hc_encode_offsets_batch(const hc_item *items, uint32_t count, uint32_t block_size, uint32_t sub_block,
                                  void *d_ws, uint64_t ws_bytes, uint32_t *d_err, void *stream);
hc_status hc_encode_pack_batch(const hc_item *items, uint32_t count, uint32_t block_size, uint32_t sub_block,
                               void *d_ws, uint64_t ws_bytes, uint32_t *d_err, void *stream);

/* hc_decode_blocks for every item (uses in, in_bytes, n, cb, block_off,   */
/* sub_idx, out).  One launch per code class present: items whose code is  */
/* a complete 8-bit code (all 256 bytes, 8 bits each) decode as a          */
/* byte-swapped copy; the rest by the table decoder, one launch for each   */
/* longest-code class (<= 8, <= 10, <= 12, <= 16, <= 24 bits, longer).     */
/* Side by side: with more than one class, the launches after the first   */
/* go to library-owned streams (default priority, created once per device) */
/* that wait for everything 'stream' holds when the call is made, and     */
/* 'stream' then waits for them, so the call is still one step in the     */
/* caller's stream order.  While 'stream' is captured into a graph the    */
/* launches run in stream order instead.  The batch encode calls do the   */
/* same with their classes.                                                */
/* Errors returned: INVALID_ARG, NO_SPACE, HIP; in *d_err: CORRUPT,         */
/* TABLE_CHANGED.                                                           */
/* Graph capture: the batch calls choose kernel variants and shapes from   */
/* every item's code (longest code, complete 8-bit code or not) when they  */
/* are called.  A captured graph therefore stays valid only while no       */
/* item's longest code grows and no complete 8-bit code stops being one    */
/* (encode and decode launch them apart); the kernels of a replay that     */
/* meet such tables leave at once and report TABLE_CHANGED in *d_err       */
/* (outputs unspecified, as after any error); shorter codes are fine.      */
hc_status hc_decode_batch(const hc_item *items, uint32_t count, uint32_t block_size, uint32_t sub_block,
                          void *d_ws, uint64_t ws_bytes, uint32_t *d_err, void *stream);

/* ---------------------------------------------------------------------- */
/* Block decoding without the sub-block index (section 2.1: a code stream  */
/* cut at fixed bit positions decodes wrongly from the cut, and Huffman    */
/* codes tend to resynchronise).  One work-group per block cuts the        */
/* block's payload into up to 256 equal pieces, decodes them all from      */
/* their first bit, then re-decodes each piece from where its left         */
/* neighbour's codes end until no start moves (at most one round per       */
/* piece), places the pieces' symbols by a scan of their counts and        */
/* decodes them into d_out.  For blocks too large for one lane each when   */
/* the encoder wrote no index (any paper-format stream).                   */
/* Arguments and layout as hc_decode_blocks with d_sub_idx = NULL: d_in    */
/* (16-byte aligned, in_bytes % 4 == 0), n, block_size, cb, d_block_off    */
/* (nb + 1 u64), d_out (n bytes, 16-byte aligned, caller-owned), d_err.    */
/* Decoding is as strict as hc_decode_blocks: CORRUPT in *d_err for an     */
/* invalid code, codes not ending exactly at the header's bit count, a     */
/* symbol count other than the block's, non-zero pad, or headers that      */
/* disagree with the offsets.  No workspace, no allocation; one launch.    */
/* Errors returned: INVALID_ARG, HIP.                                      */
/* ---------------------------------------------------------------------- */
hc_status hc_decode_blocks_selfsync(const uint8_t *d_in, uint64_t in_bytes, uint64_t n, uint32_t block_size,
                                    hc_cb_handle cb, const uint64_t *d_block_off, uint8_t *d_out, uint32_t *d_err,
                                    void *stream);

/* hc_decode_blocks_selfsync for every item (uses in, in_bytes, n, cb,     */
/* block_off, out; sub_idx is not read): the blocks of all items in one    */
/* launch per code class, one work-group per block.  Items whose code is a */
/* complete 8-bit code decode as a byte-swapped copy (every code 8 bits:   */
/* no index needed) in a launch of their own.  Workspace as               */
/* hc_decode_batch (256-byte aligned device memory of at least            */
/* hc_batch_workspace_bytes, holding the job tables; the call copies them */
/* asynchronously from the library's pinned staging ring).                 */
/* Errors returned: INVALID_ARG, NO_SPACE, HIP; in *d_err: CORRUPT,         */
/* TABLE_CHANGED (graph replays: as hc_decode_batch).                      */
hc_status hc_decode_batch_selfsync(const hc_item *items, uint32_t count, uint32_t block_size, void *d_ws,
                                   uint64_t ws_bytes, uint32_t *d_err, void *stream);

/* ---------------------------------------------------------------------- */
/* Streaming copy by a kernel of one work-group per CU, for moves between  */
/* device memory and pinned host memory that should not wait on the        */
/* runtime's copy engines (the host-resident pipeline's copy-out).         */
/* d_dst[0 .. n-1] = d_src[0 .. n-1]; both 16-byte aligned, n % 16 == 0,    */
/* no overlap.  Each range must lie inside one allocation that the device */
/* reaches at its own addresses: device memory or host memory pinned by   */
/* the HIP runtime; the call checks this with the runtime and refuses      */
/* otherwise (pageable host memory, a range running past its allocation).  */
/* One launch, no allocation.                                              */
/* Errors returned: INVALID_ARG, HIP.                                      */
/* ---------------------------------------------------------------------- */
hc_status hc_copy(const void *d_src, void *d_dst, uint64_t n, void *stream);

/* ---------------------------------------------------------------------- */
/* Roofline probes (measurement helpers, not part of the coding path):     */
/* the HBM rate plain streaming kernels reach on the device, against       */
/* which the codec kernels' rates are read.                                */
/* hc_probe_copy: d_dst[0 .. n-1] = d_src[0 .. n-1]; reads n bytes and     */
/*   writes n bytes.  Both 16-byte aligned, the ranges must not overlap.   */
/* hc_probe_read: reads d_src[0 .. n-1] (16-byte aligned) and xors its     */
/*   32-bit words into *d_sink (one u32, 4-byte aligned, caller-owned;     */
/*   the value only keeps the reads from being removed).                   */
/* n must be a multiple of 16 (n == 0: nothing is launched).  One launch   */
/* on the stream, no allocation.                                          */
/* Errors returned: INVALID_ARG (null, misaligned or overlapping           */
/* pointers, n % 16 != 0), HIP.                                            */
/* ---------------------------------------------------------------------- */
hc_status hc_probe_copy(const void *d_src, void *d_dst, uint64_t n, void *stream);
hc_status hc_probe_read(const void *d_src, uint64_t n, uint32_t *d_sink, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HC_H */
