"""CPU oracle for block-decomposed Huffman coding -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product (the HIP library and its
Python binding) never imports, links or calls it, and the oracle never imports
the product: the two share no code.

The arithmetic lives in ``hc_oracle.c`` (plain C, one bit at a time); this
module compiles it with gcc and wraps it with numpy arrays.  Each wrapper names
the passage of the paper it follows:

* ``histogram``      -- symbol counting (section 2)
* ``code_lengths``   -- Huffman tree depths, heap with a fixed tie-break (section 2, Fig. 2)
* ``canonical_codes``-- canonical code values for those lengths (RFC 1951, section 3.2.2)
* ``block_bits``     -- the length pass over each block (section 2.1)
* ``encode``         -- header + MSB-first payload + zero pad per block (section 2.1, Fig. 3-4)
* ``sub_index``      -- bit position of every S-th symbol of a block (extension of the offset table)
* ``walk``           -- offset table rebuilt from the length delimiters (section 2.1)
* ``decode``         -- strict bit-serial decode of every block (sections 2.1 and 3.2)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_hc.so")

OK = 0
ERR_INVALID_ARG = 1
ERR_NO_SPACE = 2
ERR_SYMBOL_ABSENT = 4
ERR_BLOCK_OVERFLOW = 5
ERR_CORRUPT = 6
ERR_CODE_TOO_LONG = 7


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"oracle {what} failed with status {status}")
        self.status = status


def build(force: bool = False) -> str:
    """Compile hc_oracle.c into liboracle_hc.so with gcc (plain -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC", _SRC, "-o", tmp]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64 = ctypes.c_uint64
        lib.or_histogram.argtypes = [u8p, u64, u64p]
        lib.or_histogram.restype = None
        lib.or_code_lengths.argtypes = [u64p, u8p]
        lib.or_code_lengths.restype = ctypes.c_int
        lib.or_canonical_codes.argtypes = [u8p, u64p]
        lib.or_canonical_codes.restype = ctypes.c_int
        lib.or_block_bits.argtypes = [u8p, u64, u64, u8p, u64p]
        lib.or_block_bits.restype = ctypes.c_int
        lib.or_encoded_size.argtypes = [u8p, u64, u64, u8p]
        lib.or_encoded_size.restype = u64
        lib.or_encode.argtypes = [u8p, u64, u64, u8p, u64p, u8p, u64, u64p, u64p]
        lib.or_encode.restype = ctypes.c_int
        lib.or_sub_index.argtypes = [u8p, u64, u64, u64, u8p, u32p]
        lib.or_sub_index.restype = ctypes.c_int
        lib.or_walk.argtypes = [u8p, u64, u64, u64p]
        lib.or_walk.restype = ctypes.c_int
        lib.or_decode.argtypes = [u8p, u64, u64, u64, u8p, u8p]
        lib.or_decode.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _u8(x) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(x, dtype=np.uint8).reshape(-1))
    if a.size == 0:  # keep a valid pointer for empty inputs
        return np.zeros(1, dtype=np.uint8)[:0]
    return a


def num_blocks(n: int, B: int) -> int:
    return (n + B - 1) // B


def histogram(x) -> np.ndarray:
    """h[v] = number of bytes equal to v (section 2)."""
    x = _u8(x)
    h = np.zeros(256, dtype=np.uint64)
    _load().or_histogram(_p(x, ctypes.c_uint8), x.size, _p(h, ctypes.c_uint64))
    return h


def code_lengths(hist) -> np.ndarray:
    """Huffman code lengths, merge order fixed by (weight, key) (section 2, Fig. 2)."""
    h = np.ascontiguousarray(np.asarray(hist, dtype=np.uint64).reshape(256))
    L = np.zeros(256, dtype=np.uint8)
    st = _load().or_code_lengths(_p(h, ctypes.c_uint64), _p(L, ctypes.c_uint8))
    if st != OK:
        raise OracleError(st, "code_lengths")
    return L


def canonical_codes(lengths) -> np.ndarray:
    """Canonical code values (right-aligned) for the given lengths."""
    L = np.ascontiguousarray(np.asarray(lengths, dtype=np.uint8).reshape(256))
    c = np.zeros(256, dtype=np.uint64)
    st = _load().or_canonical_codes(_p(L, ctypes.c_uint8), _p(c, ctypes.c_uint64))
    if st != OK:
        raise OracleError(st, "canonical_codes")
    return c


def codebook(hist):
    """(lengths, codes) of the oracle's Huffman code for a histogram."""
    L = code_lengths(hist)
    return L, canonical_codes(L)


def block_bits(x, B: int, lengths) -> np.ndarray:
    """Per-block payload bit counts: the length pass of section 2.1."""
    x = _u8(x)
    L = np.ascontiguousarray(np.asarray(lengths, dtype=np.uint8).reshape(256))
    nb = num_blocks(x.size, B)
    bits = np.zeros(max(nb, 1), dtype=np.uint64)
    st = _load().or_block_bits(_p(x, ctypes.c_uint8), x.size, B, _p(L, ctypes.c_uint8),
                               _p(bits, ctypes.c_uint64))
    if st != OK:
        raise OracleError(st, "block_bits")
    return bits[:nb]


def encode(x, B: int, lengths, codes):
    """Block encoder of section 2.1.  Returns (stream, offsets[nb+1], bits[nb])."""
    x = _u8(x)
    L = np.ascontiguousarray(np.asarray(lengths, dtype=np.uint8).reshape(256))
    c = np.ascontiguousarray(np.asarray(codes, dtype=np.uint64).reshape(256))
    lib = _load()
    nb = num_blocks(x.size, B)
    bits = block_bits(x, B, L)
    size = int(sum(4 + 4 * ((int(b) + 31) // 32) for b in bits))
    out = np.zeros(max(size, 1), dtype=np.uint8)
    offsets = np.zeros(nb + 1, dtype=np.uint64)
    bits2 = np.zeros(max(nb, 1), dtype=np.uint64)
    st = lib.or_encode(_p(x, ctypes.c_uint8), x.size, B, _p(L, ctypes.c_uint8), _p(c, ctypes.c_uint64),
                       _p(out, ctypes.c_uint8), out.size, _p(offsets, ctypes.c_uint64),
                       _p(bits2, ctypes.c_uint64))
    if st != OK:
        raise OracleError(st, "encode")
    return out[:size], offsets, bits2[:nb]


def sub_index(x, B: int, S: int, lengths) -> np.ndarray:
    """Bit position of symbol c*S in each block (block's bit count past its end)."""
    x = _u8(x)
    L = np.ascontiguousarray(np.asarray(lengths, dtype=np.uint8).reshape(256))
    nb = num_blocks(x.size, B)
    cpb = (B + S - 1) // S
    idx = np.zeros(max(nb * cpb, 1), dtype=np.uint32)
    st = _load().or_sub_index(_p(x, ctypes.c_uint8), x.size, B, S, _p(L, ctypes.c_uint8),
                              _p(idx, ctypes.c_uint32))
    if st != OK:
        raise OracleError(st, "sub_index")
    return idx[: nb * cpb]


def walk(stream, nb: int) -> np.ndarray:
    """Offset table rebuilt from the block headers (section 2.1)."""
    s = _u8(stream)
    offsets = np.zeros(nb + 1, dtype=np.uint64)
    st = _load().or_walk(_p(s, ctypes.c_uint8), s.size, nb, _p(offsets, ctypes.c_uint64))
    if st != OK:
        raise OracleError(st, "walk")
    return offsets


def decode_status(stream, n: int, B: int, lengths):
    """Strict decode; returns (status, output).  Output is undefined on error."""
    s = _u8(stream)
    L = np.ascontiguousarray(np.asarray(lengths, dtype=np.uint8).reshape(256))
    out = np.zeros(max(n, 1), dtype=np.uint8)
    st = _load().or_decode(_p(s, ctypes.c_uint8), s.size, n, B, _p(L, ctypes.c_uint8),
                           _p(out, ctypes.c_uint8))
    return st, out[:n]


def decode(stream, n: int, B: int, lengths) -> np.ndarray:
    """Strict decode of sections 2.1 and 3.2; raises OracleError on a bad stream."""
    st, out = decode_status(stream, n, B, lengths)
    if st != OK:
        raise OracleError(st, "decode")
    return out
