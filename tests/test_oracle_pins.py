"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself: every expected value comes from
an independent formulation (bincount, heapq Huffman, exhaustive search, string
concatenation of code words, a published worked example) or from a closed form.
"""
import heapq
import itertools
import math
import os
import struct

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ helpers
def heapq_huffman_cost(hist):
    """Textbook Huffman (any tie-break): cost = sum of all merged weights."""
    w = [int(v) for v in hist if v > 0]
    if len(w) <= 1:
        return sum(w)  # a lone symbol costs one bit per occurrence
    heap = [(v, i) for i, v in enumerate(w)]
    heapq.heapify(heap)
    counter = len(w)
    cost = 0
    while len(heap) > 1:
        a, _ = heapq.heappop(heap)
        b, _ = heapq.heappop(heap)
        cost += a + b
        heapq.heappush(heap, (a + b, counter))
        counter += 1
    return cost


def tie_break_lengths_by_sorting(hist):
    """The merge rule written out as: sort all live nodes by (weight, key) and
    merge the first two; leaf keys are symbol values, the t-th merged node gets
    key 256 + t.  Quadratic, and independent of any heap."""
    nodes = [(int(h), v, [v]) for v, h in enumerate(hist) if h > 0]
    lengths = [0] * 256
    if len(nodes) == 1:
        lengths[nodes[0][1]] = 1
        return lengths
    t = 0
    while len(nodes) > 1:
        nodes.sort(key=lambda nd: (nd[0], nd[1]))
        a, b = nodes[0], nodes[1]
        for v in a[2] + b[2]:
            lengths[v] += 1
        nodes = nodes[2:] + [(a[0] + b[0], 256 + t, a[2] + b[2])]
        t += 1
    return lengths


def bitstring(x, lengths, codes):
    return "".join(format(int(codes[v]), "0%db" % int(lengths[v])) for v in np.asarray(x).tolist())


def words_le_msb_first(bits: str) -> bytes:
    bits = bits + "0" * ((-len(bits)) % 32)
    return b"".join(struct.pack("<I", int(bits[k:k + 32], 2)) for k in range(0, len(bits), 32))


def expected_stream(x, B, lengths, codes) -> bytes:
    """The block format built from strings: per block a little-endian u32 with
    the payload bit count, then the concatenated code words packed MSB first
    into little-endian 32-bit words with zero pad."""
    x = np.asarray(x, dtype=np.uint8)
    out = b""
    for a in range(0, x.size, B):
        s = bitstring(x[a:a + B], lengths, codes)
        out += struct.pack("<I", len(s)) + words_le_msb_first(s)
    return out


def kraft_sum_scaled(lengths):
    L = [int(v) for v in lengths if v > 0]
    M = max(L)
    return sum(1 << (M - v) for v in L), 1 << M


# ------------------------------------------------------------------ histogram
def test_histogram_matches_bincount(oracle):
    x = synth.zipf_bytes(100_003, 1.2, 5)
    h = oracle.histogram(x)
    assert np.array_equal(h, np.bincount(x, minlength=256).astype(np.uint64))
    assert int(h.sum()) == x.size


def test_histogram_empty(oracle):
    assert not oracle.histogram(np.zeros(0, np.uint8)).any()


# ------------------------------------------------------------------ code lengths
def test_lengths_empty_and_single(oracle):
    assert not oracle.code_lengths(np.zeros(256, np.uint64)).any()
    h = np.zeros(256, np.uint64)
    h[77] = 12345
    L = oracle.code_lengths(h)
    assert L[77] == 1 and int(L.sum()) == 1


@pytest.mark.parametrize("seed", range(40))
def test_lengths_kraft_equality_and_optimal_cost(oracle, seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(2, 257))
    h = np.zeros(256, np.uint64)
    syms = rng.choice(256, size=m, replace=False)
    h[syms] = rng.integers(1, [10, 1000, 10**9][seed % 3], size=m).astype(np.uint64)
    L = oracle.code_lengths(h)
    assert np.array_equal(L > 0, h > 0)
    num, den = kraft_sum_scaled(L)
    assert num == den  # a full binary tree: Kraft equality
    cost = int(np.sum(h.astype(object) * L.astype(object)))
    assert cost == heapq_huffman_cost(h)


@pytest.mark.parametrize("m", [2, 3, 4, 5, 6])
def test_lengths_bruteforce_optimal(oracle, m):
    rng = np.random.default_rng(100 + m)
    for trial in range(25):
        w = rng.integers(1, 30, size=m)
        h = np.zeros(256, np.uint64)
        h[:m] = w
        L = oracle.code_lengths(h)
        best = None
        for cand in itertools.product(range(1, m), repeat=m):
            if sum(2.0 ** -c for c in cand) <= 1.0 + 1e-12:
                c = int(np.dot(w, cand))
                best = c if best is None else min(best, c)
        assert int(np.dot(w, L[:m].astype(np.int64))) == best


def test_lengths_entropy_bound(oracle):
    x = synth.zipf_bytes(1 << 20, 1.2, 9)
    h = oracle.histogram(x)
    L = oracle.code_lengths(h)
    n = x.size
    p = h[h > 0].astype(np.float64) / n
    H = float(-(p * np.log2(p)).sum())
    cost = float(np.sum(h.astype(np.float64) * L))
    assert n * H <= cost + 1e-6 < n * (H + 1)


def test_lengths_closed_forms(oracle):
    # dyadic probabilities: length = -log2 p
    h = np.zeros(256, np.uint64)
    h[[3, 9, 40, 41]] = [8, 4, 2, 2]
    L = oracle.code_lengths(h)
    assert (L[3], L[9], L[40], L[41]) == (1, 2, 3, 3)
    # 2**k equal counts: all lengths k
    for k in range(1, 9):
        h = np.zeros(256, np.uint64)
        h[: 1 << k] = 7
        L = oracle.code_lengths(h)
        assert set(L[: 1 << k].tolist()) == {k} and not L[1 << k:].any()
    # Fibonacci weights 1,1,2,3,5,...: lengths m-1, m-1, m-2, ..., 1
    for m in (3, 10, 30, 60):
        fib = [1, 1]
        while len(fib) < m:
            fib.append(fib[-1] + fib[-2])
        h = np.zeros(256, np.uint64)
        h[:m] = fib
        L = oracle.code_lengths(h)
        assert L[:m].tolist() == [m - 1] + list(range(m - 1, 0, -1))


def test_lengths_too_deep_and_overflow(oracle):
    fib = [1, 1]
    while len(fib) < 70:
        fib.append(fib[-1] + fib[-2])
    h = np.zeros(256, np.uint64)
    h[:70] = fib
    with pytest.raises(oracle.OracleError) as e:
        oracle.code_lengths(h)
    assert e.value.status == oracle.ERR_CODE_TOO_LONG
    h = np.zeros(256, np.uint64)
    h[0] = h[1] = np.uint64(1 << 63)
    with pytest.raises(oracle.OracleError) as e:
        oracle.code_lengths(h)
    assert e.value.status == oracle.ERR_INVALID_ARG


def test_lengths_monotone_in_frequency(oracle):
    x = synth.zipf_bytes(300_000, 1.1, 3)
    h = oracle.histogram(x)
    L = oracle.code_lengths(h)
    present = np.nonzero(h)[0]
    for a in present:
        for b in present:
            if h[a] > h[b]:
                assert L[a] <= L[b]


@pytest.mark.parametrize("seed", range(300))
def test_lengths_tie_break_rule(oracle, seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(1, 40 if seed % 2 else 257))
    h = np.zeros(256, np.uint64)
    syms = rng.choice(256, size=m, replace=False)
    h[syms] = rng.integers(1, [2, 3, 5, 9][seed % 4], size=m).astype(np.uint64)  # tie heavy
    assert oracle.code_lengths(h).tolist() == tie_break_lengths_by_sorting(h)


# ------------------------------------------------------------------ canonical codes
def test_canonical_rfc1951_example(oracle):
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "rfc1951_canonical_example.txt"))
            if ln.strip() and not ln.startswith("#")]
    L = np.zeros(256, np.uint8)
    for i, (_, ln, _) in enumerate(rows):
        L[i] = int(ln)
    codes = oracle.canonical_codes(L)
    for i, (_, ln, code) in enumerate(rows):
        assert format(int(codes[i]), "0%sb" % ln) == code


@pytest.mark.parametrize("seed", range(20))
def test_canonical_prefix_free_and_ordered(oracle, seed):
    rng = np.random.default_rng(seed)
    h = np.zeros(256, np.uint64)
    m = int(rng.integers(2, 257))
    h[rng.choice(256, size=m, replace=False)] = rng.integers(1, 10**6, size=m).astype(np.uint64)
    L = oracle.code_lengths(h)
    C = oracle.canonical_codes(L)
    present = [v for v in range(256) if L[v]]
    strings = {v: format(int(C[v]), "0%db" % L[v]) for v in present}
    for a in present:
        for b in present:
            if a != b:
                assert not strings[b].startswith(strings[a])
            if a < b and L[a] == L[b]:
                assert C[a] < C[b]
    M = int(L.max())
    longest = [v for v in present if L[v] == M]
    assert int(C[longest[-1]]) == (1 << M) - 1
    shortest = [v for v in present if L[v] == L[present].min()]
    assert int(C[shortest[0]]) == 0


def test_canonical_64_bit_codes(oracle):
    fib = [1, 1]
    while len(fib) < 65:
        fib.append(fib[-1] + fib[-2])
    h = np.zeros(256, np.uint64)
    h[:65] = fib
    L = oracle.code_lengths(h)
    assert int(L.max()) == 64
    C = oracle.canonical_codes(L)
    assert int(C[0]) == (1 << 64) - 2 and int(C[1]) == (1 << 64) - 1
    assert int(C[64]) == 0


# ------------------------------------------------------------------ block format
@pytest.mark.parametrize("n,B", [(1, 16), (100, 16), (4096, 4096), (10_000, 4096), (65_537, 1000),
                                 (50_000, 50_000), (50_000, 10**6)])
def test_format_closed_forms(oracle, n, B):
    x = synth.zipf_bytes(n, 1.2, n)
    h = oracle.histogram(x)
    L, C = oracle.codebook(h)
    stream, off, bits = oracle.encode(x, B, L, C)
    nb = (n + B - 1) // B
    assert off.size == nb + 1 and int(off[0]) == 0 and int(off[-1]) == stream.size
    bytes_i = np.diff(off.astype(np.int64))
    assert np.array_equal(bytes_i, 4 + 4 * ((bits.astype(np.int64) + 31) // 32))
    # compressed bit count = sum freq * len
    assert int(bits.sum()) == int(np.sum(h.astype(np.int64) * L.astype(np.int64)))
    # headers hold the bit counts
    for i in range(nb):
        assert struct.unpack_from("<I", stream.tobytes(), int(off[i]))[0] == int(bits[i])
    # per-block overhead 32..63 bits, exactly 32 iff the payload fills whole words (section 2.1)
    over = 8 * bytes_i - bits.astype(np.int64)
    assert ((over >= 32) & (over <= 63)).all()
    assert np.array_equal(over == 32, bits % 32 == 0)
    assert stream.tobytes() == expected_stream(x, B, L, C)


def test_format_single_block_is_plain_huffman(oracle):
    x = synth.zipf_bytes(20_000, 1.1, 77)
    L, C = oracle.codebook(oracle.histogram(x))
    stream, off, bits = oracle.encode(x, 1 << 20, L, C)
    plain = bitstring(x, L, C)
    assert int(bits[0]) == len(plain)
    assert stream.tobytes()[4:] == words_le_msb_first(plain)


def test_format_blocks_independent(oracle):
    x = synth.zipf_bytes(33_333, 1.3, 2)
    L, C = oracle.codebook(oracle.histogram(x))
    B = 1024
    stream, off, _ = oracle.encode(x, B, L, C)
    parts = [oracle.encode(x[a:a + B], B, L, C)[0].tobytes() for a in range(0, x.size, B)]
    assert stream.tobytes() == b"".join(parts)
    for i, a in enumerate(range(0, x.size, B)):
        blk = stream[int(off[i]):int(off[i + 1])]
        assert np.array_equal(oracle.decode(blk, min(B, x.size - a), B, L), x[a:a + B])


def test_format_exhaustive_tiny(oracle):
    # all inputs of length <= 8 over the alphabet {10, 20, 30}, four block sizes
    for n in range(1, 9):
        for tup in itertools.product((10, 20, 30), repeat=n):
            x = np.array(tup, dtype=np.uint8)
            L, C = oracle.codebook(oracle.histogram(x))
            for B in (1, 2, 3, 8):
                stream, off, bits = oracle.encode(x, B, L, C)
                assert stream.tobytes() == expected_stream(x, B, L, C)
                assert np.array_equal(oracle.decode(stream, n, B, L), x)


def test_uncompressed_ascii_is_eight_bits_per_character():
    # Fig. 1: a nine-character ASCII string occupies 72 bits before coding.
    assert np.frombuffer(b"ABCDEFGHI", dtype=np.uint8).nbytes * 8 == 72


def test_empty_input(oracle):
    L = np.zeros(256, np.uint8)
    L[0] = 1
    stream, off, bits = oracle.encode(np.zeros(0, np.uint8), 4096, L, oracle.canonical_codes(L))
    assert stream.size == 0 and off.tolist() == [0] and bits.size == 0
    assert oracle.decode(stream, 0, 4096, L).size == 0


@settings(max_examples=60, deadline=None)
@given(n=st.integers(0, 3000), B=st.integers(1, 700), s=st.floats(0.5, 3.0), seed=st.integers(0, 2**31))
def test_round_trip_property(oracle, n, B, s, seed):
    x = synth.zipf_bytes(n, s, seed)
    L, C = oracle.codebook(oracle.histogram(x))
    if n == 0:
        L[0] = 1
        C = oracle.canonical_codes(L)
    stream, off, bits = oracle.encode(x, B, L, C)
    assert np.array_equal(oracle.decode(stream, n, B, L), x)
    assert np.array_equal(oracle.walk(stream, (n + B - 1) // B), off)


def test_sub_index_is_prefix_of_lengths(oracle):
    x = synth.zipf_bytes(10_000, 1.2, 4)
    L, C = oracle.codebook(oracle.histogram(x))
    B, S = 4096, 1024
    idx = oracle.sub_index(x, B, S, L).reshape(-1, 4)
    lens = L[x].astype(np.int64)
    for i, a in enumerate(range(0, x.size, B)):
        blk = lens[a:a + B]
        csum = np.concatenate([[0], np.cumsum(blk)])
        for c in range(4):
            k = min(c * S, blk.size)
            assert int(idx[i, c]) == int(csum[k])


# ------------------------------------------------------------------ strict decoding
def _valid(oracle, n=5000, B=512, seed=1):
    x = synth.zipf_bytes(n, 1.2, seed)
    L, C = oracle.codebook(oracle.histogram(x))
    stream, off, bits = oracle.encode(x, B, L, C)
    return x, L, C, stream.copy(), off, bits


def test_corrupt_header_bit(oracle):
    x, L, C, s, off, bits = _valid(oracle)
    s[int(off[3])] ^= 0x01  # odd/even bit count change moves the block's end
    st_, _ = oracle.decode_status(s, x.size, 512, L)
    assert st_ == oracle.ERR_CORRUPT


def test_corrupt_header_too_large(oracle):
    x, L, C, s, off, bits = _valid(oracle)
    s[int(off[-2]) + 3] = 0x7F
    assert oracle.decode_status(s, x.size, 512, L)[0] == oracle.ERR_CORRUPT
    with pytest.raises(oracle.OracleError):
        oracle.walk(s, off.size - 1)


def test_corrupt_nonzero_pad(oracle):
    x, L, C, s, off, bits = _valid(oracle)
    i = next(i for i in range(bits.size) if bits[i] % 32 != 0)
    pad_bit = int(bits[i])  # first pad bit of block i
    word = int(off[i]) + 4 + 4 * (pad_bit // 32)
    pos = 31 - pad_bit % 32
    s[word + pos // 8] |= 1 << (pos % 8)
    assert oracle.decode_status(s, x.size, 512, L)[0] == oracle.ERR_CORRUPT


def test_corrupt_truncated_and_trailing(oracle):
    x, L, C, s, off, bits = _valid(oracle)
    assert oracle.decode_status(s[:-4], x.size, 512, L)[0] == oracle.ERR_CORRUPT
    assert oracle.decode_status(np.concatenate([s, np.zeros(4, np.uint8)]), x.size, 512, L)[0] \
        == oracle.ERR_CORRUPT
    # wrong symbol count: one more block than the stream holds, or one block fewer
    assert oracle.decode_status(s, x.size + 512, 512, L)[0] == oracle.ERR_CORRUPT
    assert oracle.decode_status(s, x.size - 1024, 512, L)[0] == oracle.ERR_CORRUPT


def test_corrupt_invalid_code_foreign_codebook(oracle):
    # an incomplete code (Kraft sum < 1) leaves bit patterns that are no code
    L = np.zeros(256, np.uint8)
    L[[1, 2]] = [1, 2]  # codes 0 and 10; "11" is invalid
    C = oracle.canonical_codes(L)
    x = np.array([1, 2, 1, 1], np.uint8)
    s, off, bits = oracle.encode(x, 16, L, C)
    assert np.array_equal(oracle.decode(s, 4, 16, L), x)
    s = s.copy()
    s[4 + 3] |= 0xC0  # payload begins with "11"
    assert oracle.decode_status(s, 4, 16, L)[0] == oracle.ERR_CORRUPT


def test_symbol_absent(oracle):
    L = np.zeros(256, np.uint8)
    L[[1, 2]] = 1
    C = oracle.canonical_codes(L)
    with pytest.raises(oracle.OracleError) as e:
        oracle.encode(np.array([1, 2, 3], np.uint8), 16, L, C)
    assert e.value.status == oracle.ERR_SYMBOL_ABSENT
