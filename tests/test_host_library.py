"""CPU-side checks of libhc.so: exported symbols, host code construction
against the oracle, host-detected argument errors.  No GPU is touched."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hc.h")


@pytest.fixture(scope="module")
def hc():
    import paper_1107_1525_amd as hc_mod

    return hc_mod


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hc_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol(hc):
    names = declared_functions()
    assert len(names) >= 12
    lib = ctypes.CDLL(hc.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings(hc):
    assert hc.hc_status_str(0) == "HC_OK"
    assert hc.hc_status_str(6) == "HC_ERR_CORRUPT"
    assert hc.hc_status_str(99) == "HC_ERR_UNKNOWN"


@pytest.mark.parametrize("seed", range(2000))
def test_two_queue_matches_heap_tie_break(hc, oracle, seed):
    """The library's two-queue Huffman and the oracle's heap apply the same
    (weight, key) merge order, so their lengths agree exactly, ties included."""
    rng = np.random.default_rng(seed)
    kind = seed % 5
    h = np.zeros(256, np.uint64)
    m = int(rng.integers(1, 257))
    syms = rng.choice(256, size=m, replace=False)
    if kind == 0:
        h[syms] = rng.integers(1, 3, size=m)            # massive ties
    elif kind == 1:
        h[syms] = rng.integers(1, 1 << 40, size=m)      # wide weights
    elif kind == 2:
        h[syms] = 2 ** rng.integers(0, 20, size=m)      # dyadic, tie heavy
    elif kind == 3:
        h[syms] = rng.integers(1, 6, size=m) * 1000
    else:
        x = synth.zipf_bytes(int(rng.integers(1, 5000)), float(rng.uniform(0.5, 2.5)), seed)
        h = np.bincount(x, minlength=256).astype(np.uint64)
    cb = hc.hc_build_codebook(h)
    L_or = oracle.code_lengths(h)
    assert np.array_equal(cb.lengths, L_or)
    assert np.array_equal(cb.codes, oracle.canonical_codes(L_or))
    assert cb.max_len == int(L_or.max()) and cb.nsym == int((h > 0).sum())


def test_two_queue_matches_heap_1e5_histograms(hc, oracle):
    """10^5 more histograms, random and adversarial (ties, wide and dyadic
    weights, few symbols, one symbol): the library's two-queue build and the
    oracle's heap give the same lengths every time."""
    rng = np.random.default_rng(1107)
    for k in range(100_000):
        kind = k % 6
        h = np.zeros(256, np.uint64)
        m = int(rng.integers(1, 257)) if kind < 4 else int(rng.integers(1, 9))
        syms = rng.choice(256, size=m, replace=False)
        if kind == 0:
            h[syms] = rng.integers(1, 3, size=m)
        elif kind == 1:
            h[syms] = rng.integers(1, 1 << 40, size=m)
        elif kind == 2:
            h[syms] = 2 ** rng.integers(0, 30, size=m)
        elif kind == 3:
            h[syms] = rng.integers(1, 1 << 16, size=m)
        else:  # few symbols: every tie pattern of small alphabets comes up
            h[syms] = rng.integers(1, 4, size=m)
        L_or = oracle.code_lengths(h)
        assert np.array_equal(hc.hc_build_codebook(h).lengths, L_or), k


def test_codebook_fibonacci_depth(hc, oracle):
    fib = [1, 1]
    while len(fib) < 65:
        fib.append(fib[-1] + fib[-2])
    h = np.zeros(256, np.uint64)
    h[:65] = fib
    cb = hc.hc_build_codebook(h)
    assert cb.max_len == 64
    assert np.array_equal(cb.lengths, oracle.code_lengths(h))
    assert np.array_equal(cb.codes, oracle.canonical_codes(oracle.code_lengths(h)))
    fib70 = [1, 1]
    while len(fib70) < 70:
        fib70.append(fib70[-1] + fib70[-2])
    h[:70] = fib70
    with pytest.raises(hc.HcError) as e:
        hc.hc_build_codebook(h)
    assert e.value.status == hc.HC_ERR_CODE_TOO_LONG


def test_codebook_edge_cases(hc):
    cb = hc.hc_build_codebook(np.zeros(256, np.uint64))
    assert cb.max_len == 0 and cb.nsym == 0
    h = np.zeros(256, np.uint64)
    h[200] = 5
    cb = hc.hc_build_codebook(h)
    assert cb.lengths[200] == 1 and cb.codes[200] == 0 and cb.max_len == 1
    h = np.zeros(256, np.uint64)
    h[0] = h[1] = np.uint64(1 << 63)
    with pytest.raises(hc.HcError) as e:
        hc.hc_build_codebook(h)
    assert e.value.status == hc.HC_ERR_INVALID_ARG


def test_codebook_from_lengths(hc, oracle):
    L = np.zeros(256, np.uint8)
    L[[5, 6, 7]] = [1, 2, 2]
    cb = hc.hc_codebook_from_lengths(L)
    assert np.array_equal(cb.codes, oracle.canonical_codes(L))
    L[8] = 2  # Kraft sum above one
    with pytest.raises(hc.HcError):
        hc.hc_codebook_from_lengths(L)
    L = np.zeros(256, np.uint8)
    L[[1, 2]] = [1, 2]  # incomplete code is allowed
    assert np.array_equal(hc.hc_codebook_from_lengths(L).codes, oracle.canonical_codes(L))


def test_encode_bound_and_sizes(hc):
    assert hc.hc_encode_bound(0, 4096, 8) == 0
    assert hc.hc_encode_bound(4096, 4096, 8) == 4 + 4096
    assert hc.hc_encode_bound(4097, 4096, 8) == 4 + 4096 + 4 + 4
    assert hc.hc_encode_bound(100, 16, 3) == 6 * (4 + 8) + (4 + 4)
    assert hc.hc_encode_bound(10, 0, 8) == 0
    assert hc.hc_encode_bound(10, 16, 65) == 0
    assert hc.hc_sub_index_entries(10_000, 4096, 1024) == 3 * 4
    assert hc.hc_sub_index_entries(10_000, 4096, 0) == 0
    assert hc.hc_encode_workspace_bytes(1 << 20, 4096) > 0


def test_host_argument_errors(hc):
    lib = ctypes.CDLL(hc.LIB_PATH)
    vp = ctypes.c_void_p
    lib.hc_histogram.argtypes = [vp, ctypes.c_uint64, vp, vp]
    assert lib.hc_histogram(None, 10, None, None) == hc.HC_ERR_INVALID_ARG
    assert lib.hc_histogram(vp(16), 10, vp(12), None) == hc.HC_ERR_INVALID_ARG  # misaligned d_hist
    assert lib.hc_histogram(vp(8), 10, vp(16), None) == hc.HC_ERR_INVALID_ARG   # misaligned d_in
    u64, u32 = ctypes.c_uint64, ctypes.c_uint32
    lib.hc_probe_copy.argtypes = [vp, vp, u64, vp]
    lib.hc_probe_read.argtypes = [vp, u64, vp, vp]
    assert lib.hc_probe_copy(vp(16), vp(4096), 24, None) == hc.HC_ERR_INVALID_ARG      # n % 16
    assert lib.hc_probe_copy(vp(8), vp(4096), 32, None) == hc.HC_ERR_INVALID_ARG       # misaligned src
    assert lib.hc_probe_copy(vp(4096), vp(4112), 32, None) == hc.HC_ERR_INVALID_ARG    # overlap
    assert lib.hc_probe_copy(None, vp(4096), 32, None) == hc.HC_ERR_INVALID_ARG
    assert lib.hc_probe_copy(None, None, 0, None) == hc.HC_OK                          # nothing to do
    assert lib.hc_probe_read(vp(16), 32, None, None) == hc.HC_ERR_INVALID_ARG          # no sink
    assert lib.hc_probe_read(vp(16), 32, vp(4098), None) == hc.HC_ERR_INVALID_ARG      # misaligned sink
    assert lib.hc_probe_read(vp(24), 32, vp(4096), None) == hc.HC_ERR_INVALID_ARG      # misaligned src
    lib.hc_encode_blocks.argtypes = [vp, u64, u32, vp, vp, u64, vp, vp, u32, vp, u64, vp, vp]
    for B in (0, 8, 24, (1 << 26) + 16):
        assert lib.hc_encode_blocks(vp(16), 100, B, vp(16), vp(16), 1 << 20, vp(16), None, 0, vp(16),
                                    1 << 20, None, None) == hc.HC_ERR_INVALID_ARG
    assert lib.hc_encode_blocks(vp(16), 100, 16, None, vp(16), 1 << 20, vp(16), None, 0, vp(16),
                                1 << 20, None, None) == hc.HC_ERR_INVALID_ARG  # no codebook
    assert lib.hc_encode_blocks(vp(16), 100, 16, vp(16), vp(16), 1 << 20, vp(16), vp(16), 0, vp(16),
                                1 << 20, None, None) == hc.HC_ERR_INVALID_ARG  # index without stride
    lib.hc_decode_blocks.argtypes = [vp, u64, u64, u32, vp, vp, vp, u32, vp, vp, vp]
    assert lib.hc_decode_blocks(vp(16), 64, 100, 17, vp(16), vp(16), None, 0, vp(16), None,
                                None) == hc.HC_ERR_INVALID_ARG
    assert lib.hc_decode_blocks(vp(16), 64, 100, 16, vp(16), vp(16), None, 24, vp(16), None,
                                None) == hc.HC_ERR_INVALID_ARG
    # no offset table: refused (the decode neither walks nor allocates; hc_walk_blocks first)
    assert lib.hc_decode_blocks(vp(16), 64, 100, 16, vp(16), None, None, 0, vp(16), None,
                                None) == hc.HC_ERR_INVALID_ARG
    lib.hc_decode_batch_selfsync.argtypes = [vp, u32, u32, vp, u64, vp, vp]
    assert lib.hc_decode_batch_selfsync(None, 1, 4096, vp(256), 1 << 20, None, None) == hc.HC_ERR_INVALID_ARG
    items = hc.make_items(1)
    assert lib.hc_decode_batch_selfsync(ctypes.cast(items, vp), 1, 24, vp(256), 1 << 20, None,
                                        None) == hc.HC_ERR_INVALID_ARG  # block size not a multiple of 16
    assert lib.hc_decode_batch_selfsync(ctypes.cast(items, vp), 1, 4096, vp(8), 1 << 20, None,
                                        None) == hc.HC_ERR_INVALID_ARG  # misaligned workspace
    assert lib.hc_decode_batch_selfsync(ctypes.cast(items, vp), 1, 4096, vp(256), 16, None,
                                        None) == hc.HC_ERR_NO_SPACE  # workspace too small for the job table
    lib.hc_walk_blocks.argtypes = [vp, u64, u64, vp, vp, vp]
    assert lib.hc_walk_blocks(vp(16), 10, 1, vp(16), None, None) == hc.HC_ERR_INVALID_ARG  # size % 4
