"""Python binding of libhc.so, the gfx950 block-decomposed Huffman codec.

Argument marshalling only: every step of the coding path runs in the HIP
kernels of libhc.so (or, for code construction over 256 symbols, in its host
C++).  PyTorch supplies device memory and streams.  The functions keep the
names of the C ABI in ``include/hc.h``:

    hc_histogram, hc_build_codebook, hc_codebook_from_lengths,
    hc_set_tuning, hc_get_tuning,
    hc_codebook_upload, hc_codebook_update, hc_codebook_destroy, hc_encode_bound,
    hc_encode_workspace_bytes, hc_sub_index_entries, hc_encode_blocks, hc_encode_blocks_noalloc,
    hc_walk_blocks, hc_decode_blocks, hc_status_str, hc_batch_workspace_bytes,
    hc_histogram_batch, hc_encode_batch, hc_encode_lengths_batch, hc_encode_offsets_batch,
    hc_encode_pack_batch, hc_decode_batch, hc_decode_blocks_selfsync, hc_decode_batch_selfsync,
    hc_cbset_create,
    hc_cbset_handle, hc_cbset_build, hc_cbset_destroy (as CodebookSet)

and add two conveniences, ``compress`` and ``decompress``, that chain them.
u64 device buffers are held in int64 tensors and u32 ones in int32 tensors
(same bits).  If libhc.so has not been built, importing this package fails.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch  # loads the HIP runtime that libhc.so then shares

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhc.so")

HC_OK = 0
HC_ERR_INVALID_ARG = 1
HC_ERR_NO_SPACE = 2
HC_ERR_HIP = 3
HC_ERR_SYMBOL_ABSENT = 4
HC_ERR_BLOCK_OVERFLOW = 5
HC_ERR_CORRUPT = 6
HC_ERR_CODE_TOO_LONG = 7
HC_ERR_TABLE_CHANGED = 8


class HcError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = int(status)
        super().__init__(f"{what}: {hc_status_str(status)} ({status})" if what else hc_status_str(status))


class hc_codebook(ctypes.Structure):
    _fields_ = [
        ("len", ctypes.c_uint8 * 256),
        ("code", ctypes.c_uint64 * 256),
        ("max_len", ctypes.c_uint32),
        ("nsym", ctypes.c_uint32),
    ]

    @property
    def lengths(self) -> np.ndarray:
        return np.frombuffer(bytes(self.len), dtype=np.uint8).copy()

    @property
    def codes(self) -> np.ndarray:
        return np.ctypeslib.as_array(self.code).astype(np.uint64).copy()


class hc_tuning(ctypes.Structure):
    """Process-wide launch parameters (see hc_tuning in include/hc.h)."""
    _fields_ = [("encode_tile_loads", ctypes.c_uint32)]


class hc_item(ctypes.Structure):
    """One buffer of a batch call (see hc_item in include/hc.h)."""
    _fields_ = [
        ("in_", ctypes.c_void_p),
        ("n", ctypes.c_uint64),
        ("in_bytes", ctypes.c_uint64),
        ("cb", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
        ("out_cap", ctypes.c_uint64),
        ("block_off", ctypes.c_void_p),
        ("sub_idx", ctypes.c_void_p),
        ("hist", ctypes.c_void_p),
    ]


if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python paper_1107_1525_amd/build.py` "
        "(there is no fallback path)"
    )
_lib = ctypes.CDLL(LIB_PATH)

_vp = ctypes.c_void_p
_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32
_st = ctypes.c_int
_sigs = {
    "hc_status_str": ([ctypes.c_int], ctypes.c_char_p),
    "hc_version": ([], ctypes.c_int),
    "hc_set_tuning": ([ctypes.POINTER(hc_tuning)], _st),
    "hc_get_tuning": ([ctypes.POINTER(hc_tuning)], _st),
    "hc_histogram": ([_vp, _u64, _vp, _vp], _st),
    "hc_build_codebook": ([_vp, ctypes.POINTER(hc_codebook)], _st),
    "hc_codebook_from_lengths": ([_vp, ctypes.POINTER(hc_codebook)], _st),
    "hc_codebook_upload": ([ctypes.POINTER(hc_codebook), ctypes.POINTER(_vp)], _st),
    "hc_codebook_update": ([_vp, ctypes.POINTER(hc_codebook), _vp], _st),
    "hc_codebook_destroy": ([_vp], _st),
    "hc_cbset_create": ([_u32, ctypes.POINTER(_vp)], _st),
    "hc_cbset_handle": ([_vp, _u32], _vp),
    "hc_cbset_build": ([_vp, _vp, ctypes.POINTER(hc_codebook), _vp], _st),
    "hc_cbset_destroy": ([_vp], _st),
    "hc_encode_bound": ([_u64, _u32, _u32], _u64),
    "hc_encode_workspace_bytes": ([_u64, _u32], _u64),
    "hc_sub_index_entries": ([_u64, _u32, _u32], _u64),
    "hc_encode_blocks": ([_vp, _u64, _u32, _vp, _vp, _u64, _vp, _vp, _u32, _vp, _u64, _vp, _vp], _st),
    "hc_encode_blocks_noalloc": ([_vp, _u64, _u32, _vp, _vp, _u64, _vp, _vp, _u32, _vp, _vp], _st),
    "hc_walk_blocks": ([_vp, _u64, _u64, _vp, _vp, _vp], _st),
    "hc_decode_blocks": ([_vp, _u64, _u64, _u32, _vp, _vp, _vp, _u32, _vp, _vp, _vp], _st),
    "hc_batch_workspace_bytes": ([ctypes.POINTER(hc_item), _u32, _u32], _u64),
    "hc_histogram_batch": ([ctypes.POINTER(hc_item), _u32, _vp, _u64, _vp], _st),
    "hc_encode_batch": ([ctypes.POINTER(hc_item), _u32, _u32, _u32, _vp, _u64, _vp, _vp], _st),
    "hc_encode_lengths_batch": ([ctypes.POINTER(hc_item), _u32, _u32, _u32, _vp, _u64, _vp, _vp], _st),
    "hc_encode_offsets_batch": ([ctypes.POINTER(hc_item), _u32, _u32, _u32, _vp, _u64, _vp, _vp], _st),
    "hc_encode_pack_batch": ([ctypes.POINTER(hc_item), _u32, _u32, _u32, _vp, _u64, _vp, _vp], _st),
    "hc_decode_batch": ([ctypes.POINTER(hc_item), _u32, _u32, _u32, _vp, _u64, _vp, _vp], _st),
    "hc_decode_blocks_selfsync": ([_vp, _u64, _u64, _u32, _vp, _vp, _vp, _vp, _vp], _st),
    "hc_decode_batch_selfsync": ([ctypes.POINTER(hc_item), _u32, _u32, _vp, _u64, _vp, _vp], _st),
    "hc_copy": ([_vp, _vp, _u64, _vp], _st),
    "hc_probe_copy": ([_vp, _vp, _u64, _vp], _st),
    "hc_probe_read": ([_vp, _u64, _vp, _vp], _st),
}
for _name, (_args, _res) in _sigs.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res


def hc_status_str(status: int) -> str:
    return _lib.hc_status_str(int(status)).decode()


def hc_version() -> int:
    return _lib.hc_version()


def hc_set_tuning(encode_tile_loads: int = 0) -> None:
    t = hc_tuning(encode_tile_loads)
    _check(_lib.hc_set_tuning(ctypes.byref(t)), "hc_set_tuning")


def hc_get_tuning() -> dict:
    t = hc_tuning()
    _check(_lib.hc_get_tuning(ctypes.byref(t)), "hc_get_tuning")
    return {"encode_tile_loads": int(t.encode_tile_loads)}


def _check(status: int, what: str):
    if status != HC_OK:
        raise HcError(status, what)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------------ a1: counts
def hc_histogram(x: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Symbol counts of a uint8 device tensor -> int64[256] device tensor (u64 bits)."""
    assert x.dtype == torch.uint8 and x.is_cuda and x.is_contiguous()
    if out is None:
        out = torch.empty(256, dtype=torch.int64, device=x.device)
    _check(_lib.hc_histogram(_ptr(x), x.numel(), _ptr(out), _stream(stream)), "hc_histogram")
    return out


# ------------------------------------------------------------------ a2: codebook
def hc_build_codebook(hist) -> hc_codebook:
    """Huffman lengths + canonical codes from 256 counts (host)."""
    h = np.ascontiguousarray(np.asarray(hist).astype(np.uint64).reshape(256))
    cb = hc_codebook()
    _check(_lib.hc_build_codebook(h.ctypes.data_as(_vp), ctypes.byref(cb)), "hc_build_codebook")
    return cb


def hc_codebook_from_lengths(lengths) -> hc_codebook:
    L = np.ascontiguousarray(np.asarray(lengths, dtype=np.uint8).reshape(256))
    cb = hc_codebook()
    _check(_lib.hc_codebook_from_lengths(L.ctypes.data_as(_vp), ctypes.byref(cb)), "hc_codebook_from_lengths")
    return cb


class DeviceCodebook:
    """An uploaded codebook (hc_cb_handle); freed by close() or on collection."""

    def __init__(self, cb: hc_codebook):
        self.host = cb
        self.max_len = int(cb.max_len)
        h = ctypes.c_void_p()
        _check(_lib.hc_codebook_upload(ctypes.byref(cb), ctypes.byref(h)), "hc_codebook_upload")
        self.handle = h

    def update(self, cb: hc_codebook, stream=None):
        """Asynchronous table refresh on the stream (hc_codebook_update)."""
        _check(_lib.hc_codebook_update(self.handle, ctypes.byref(cb), _stream(stream)), "hc_codebook_update")
        self.host = cb
        self.max_len = int(cb.max_len)

    def close(self):
        if self.handle:
            _check(_lib.hc_codebook_destroy(self.handle), "hc_codebook_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _SetCodebook:
    """Handle of one table of a CodebookSet; usable wherever a DeviceCodebook is."""

    def __init__(self, owner, handle_value: int):
        self._owner = owner  # keeps the set alive
        self.handle = ctypes.c_void_p(handle_value)
        self.host = hc_codebook()
        self.max_len = 0


class CodebookSet:
    """Device-resident code tables for many buffers, rebuilt together from
    their histograms with one copy (hc_cbset_*)."""

    def __init__(self, count: int):
        h = ctypes.c_void_p()
        _check(_lib.hc_cbset_create(count, ctypes.byref(h)), "hc_cbset_create")
        self._h = h
        self.count = count
        self.books = [_SetCodebook(self, _lib.hc_cbset_handle(h, k)) for k in range(count)]
        self._out = (hc_codebook * count)()

    def build(self, hists: np.ndarray, stream=None):
        """hists: (count, 256) uint64 on the host."""
        hh = np.ascontiguousarray(np.asarray(hists, dtype=np.uint64).reshape(self.count, 256))
        _check(_lib.hc_cbset_build(self._h, hh.ctypes.data_as(_vp), self._out, _stream(stream)), "hc_cbset_build")
        for k, b in enumerate(self.books):
            b.host = self._out[k]
            b.max_len = int(self._out[k].max_len)
        return self.books

    def __getitem__(self, k):
        return self.books[k]

    def close(self):
        if self._h:
            _check(_lib.hc_cbset_destroy(self._h), "hc_cbset_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hc_codebook_upload(cb: hc_codebook) -> DeviceCodebook:
    return DeviceCodebook(cb)


def hc_codebook_update(dcb: DeviceCodebook, cb: hc_codebook, stream=None):
    dcb.update(cb, stream)


def hc_codebook_destroy(dcb: DeviceCodebook):
    dcb.close()


# ------------------------------------------------------------------ a3-a5: encode
def hc_encode_bound(n: int, block_size: int, max_len: int) -> int:
    return int(_lib.hc_encode_bound(n, block_size, max_len))


def hc_encode_workspace_bytes(n: int, block_size: int) -> int:
    return int(_lib.hc_encode_workspace_bytes(n, block_size))


def hc_sub_index_entries(n: int, block_size: int, sub_block: int) -> int:
    return int(_lib.hc_sub_index_entries(n, block_size, sub_block))


def num_blocks(n: int, block_size: int) -> int:
    return (n + block_size - 1) // block_size


def hc_encode_blocks(x: torch.Tensor, block_size: int, dcb: DeviceCodebook, out: torch.Tensor,
                     block_off: torch.Tensor, sub_idx: Optional[torch.Tensor], sub_block: int,
                     ws: torch.Tensor, err: torch.Tensor, stream=None) -> None:
    """Raw call: every buffer is caller-provided (see include/hc.h)."""
    rc = _lib.hc_encode_blocks(_ptr(x), x.numel(), block_size, dcb.handle, _ptr(out), out.numel(),
                               _ptr(block_off), _ptr(sub_idx), sub_block, _ptr(ws), ws.numel(),
                               _ptr(err), _stream(stream))
    _check(rc, "hc_encode_blocks")


HC_NOALLOC_SCRATCH_BYTES = 32 << 20  # HC_NOALLOC_SCRATCH_BYTES of include/hc.h


def hc_encode_blocks_noalloc(x: torch.Tensor, block_size: int, dcb: DeviceCodebook, out: torch.Tensor,
                             block_off: torch.Tensor, sub_idx: Optional[torch.Tensor], sub_block: int,
                             err: torch.Tensor, stream=None) -> None:
    """hc_encode_blocks with the library's own per-GPU scratch (no workspace argument)."""
    rc = _lib.hc_encode_blocks_noalloc(_ptr(x), x.numel(), block_size, dcb.handle, _ptr(out), out.numel(),
                                       _ptr(block_off), _ptr(sub_idx), sub_block, _ptr(err), _stream(stream))
    _check(rc, "hc_encode_blocks_noalloc")


def hc_walk_blocks(stream_bytes: torch.Tensor, in_bytes: int, nb: int, block_off: torch.Tensor,
                   err: torch.Tensor, stream=None) -> None:
    rc = _lib.hc_walk_blocks(_ptr(stream_bytes), in_bytes, nb, _ptr(block_off), _ptr(err), _stream(stream))
    _check(rc, "hc_walk_blocks")


def hc_decode_blocks(stream_bytes: torch.Tensor, in_bytes: int, n: int, block_size: int, dcb: DeviceCodebook,
                     block_off: torch.Tensor, sub_idx: Optional[torch.Tensor], sub_block: int,
                     out: torch.Tensor, err: torch.Tensor, stream=None) -> None:
    rc = _lib.hc_decode_blocks(_ptr(stream_bytes), in_bytes, n, block_size, dcb.handle, _ptr(block_off),
                               _ptr(sub_idx), sub_block, _ptr(out), _ptr(err), _stream(stream))
    _check(rc, "hc_decode_blocks")


def hc_decode_blocks_selfsync(stream_bytes: torch.Tensor, in_bytes: int, n: int, block_size: int,
                              dcb: DeviceCodebook, block_off: torch.Tensor, out: torch.Tensor, err: torch.Tensor,
                              stream=None) -> None:
    """Block decode without the sub-block index (pieces resynchronised per block)."""
    rc = _lib.hc_decode_blocks_selfsync(_ptr(stream_bytes), in_bytes, n, block_size, dcb.handle, _ptr(block_off),
                                        _ptr(out), _ptr(err), _stream(stream))
    _check(rc, "hc_decode_blocks_selfsync")


# ------------------------------------------------------------------ conveniences
@dataclass
class Encoded:
    stream: torch.Tensor      # uint8[C] view of the output buffer
    block_off: torch.Tensor   # int64[nb + 1] (u64 offsets)
    sub_idx: Optional[torch.Tensor]  # int32[nb * ceil(B/S)] or None
    n: int
    block_size: int
    sub_block: int
    codebook: DeviceCodebook

    @property
    def nbytes(self) -> int:
        return int(self.stream.numel())


def new_error_word(device) -> torch.Tensor:
    return torch.zeros(1, dtype=torch.int32, device=device)


def read_error(err: torch.Tensor) -> int:
    return int(err.item()) & 0xFFFFFFFF


def compress(x: torch.Tensor, block_size: int, sub_block: int = 0, codebook: Optional[DeviceCodebook] = None,
             check: bool = True) -> Encoded:
    """hist -> codebook -> encode on the current stream; synchronises twice
    (histogram read-back, compressed size read-back)."""
    dev = x.device
    n = x.numel()
    if codebook is None:
        hist = hc_histogram(x).cpu().numpy().view(np.uint64)
        cb = hc_build_codebook(hist)
        if cb.max_len == 0:  # empty input: any one-symbol code
            L = np.zeros(256, np.uint8)
            L[0] = 1
            cb = hc_codebook_from_lengths(L)
        codebook = DeviceCodebook(cb)
    nb = num_blocks(n, block_size)
    cap = max(hc_encode_bound(n, block_size, codebook.max_len), 16)
    out = torch.empty((cap + 15) // 16 * 16, dtype=torch.uint8, device=dev)
    off = torch.empty(nb + 1, dtype=torch.int64, device=dev)
    sub = None
    if sub_block:
        sub = torch.empty(max(hc_sub_index_entries(n, block_size, sub_block), 1), dtype=torch.int32, device=dev)
    ws = torch.empty(max(hc_encode_workspace_bytes(n, block_size), 16), dtype=torch.uint8, device=dev)
    err = new_error_word(dev)
    hc_encode_blocks(x, block_size, codebook, out, off, sub, sub_block, ws, err)
    C = int(off[nb].item())
    if check:
        e = read_error(err)
        if e:
            raise HcError(e, "hc_encode_blocks (device)")
    return Encoded(out[:C], off, sub, n, block_size, sub_block, codebook)


def decompress(enc: Encoded, out: Optional[torch.Tensor] = None, use_offsets: bool = True,
               check: bool = True) -> torch.Tensor:
    dev = enc.stream.device
    if out is None:
        out = torch.empty(max(enc.n, 16), dtype=torch.uint8, device=dev)[: enc.n]
    err = new_error_word(dev)
    off = enc.block_off
    if not use_offsets:
        off = torch.empty_like(enc.block_off)
        hc_walk_blocks(enc.stream, enc.nbytes, num_blocks(enc.n, enc.block_size), off, err)
    hc_decode_blocks(enc.stream, enc.nbytes, enc.n, enc.block_size, enc.codebook, off, enc.sub_idx,
                     enc.sub_block, out, err)
    if check:
        e = read_error(err)
        if e:
            raise HcError(e, "hc_decode_blocks (device)")
    return out


# ------------------------------------------------------------------ batches
def make_items(count: int):
    """A zeroed hc_item array of the given length, to fill field by field."""
    return (hc_item * count)()


def _item_ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def set_item(items, k: int, x: Optional[torch.Tensor] = None, n: Optional[int] = None, in_bytes: int = 0,
             dcb: Optional[DeviceCodebook] = None, out: Optional[torch.Tensor] = None,
             block_off: Optional[torch.Tensor] = None, sub_idx: Optional[torch.Tensor] = None,
             hist: Optional[torch.Tensor] = None):
    it = items[k]
    it.in_ = _item_ptr(x)
    it.n = x.numel() if n is None else n
    it.in_bytes = in_bytes
    it.cb = dcb.handle.value if dcb is not None else None
    it.out = _item_ptr(out)
    it.out_cap = 0 if out is None else out.numel()
    it.block_off = _item_ptr(block_off)
    it.sub_idx = _item_ptr(sub_idx)
    it.hist = _item_ptr(hist)


def hc_batch_workspace_bytes(items, block_size: int) -> int:
    return int(_lib.hc_batch_workspace_bytes(items, len(items), block_size))


def hc_histogram_batch(items, ws: torch.Tensor, stream=None) -> None:
    _check(_lib.hc_histogram_batch(items, len(items), _ptr(ws), ws.numel(), _stream(stream)), "hc_histogram_batch")


def hc_encode_batch(items, block_size: int, sub_block: int, ws: torch.Tensor, err: torch.Tensor,
                    stream=None) -> None:
    _check(_lib.hc_encode_batch(items, len(items), block_size, sub_block, _ptr(ws), ws.numel(), _ptr(err),
                                _stream(stream)), "hc_encode_batch")


def hc_encode_lengths_batch(items, block_size: int, sub_block: int, ws: torch.Tensor, err: torch.Tensor,
                            stream=None) -> None:
    _check(_lib.hc_encode_lengths_batch(items, len(items), block_size, sub_block, _ptr(ws), ws.numel(), _ptr(err),
                                        _stream(stream)), "hc_encode_lengths_batch")


def hc_encode_offsets_batch(items, block_size: int, sub_block: int, ws: torch.Tensor, err: torch.Tensor,
                            stream=None) -> None:
    _check(_lib.hc_encode_offsets_batch(items, len(items), block_size, sub_block, _ptr(ws), ws.numel(), _ptr(err),
                                        _stream(stream)), "hc_encode_offsets_batch")


def hc_encode_pack_batch(items, block_size: int, sub_block: int, ws: torch.Tensor, err: torch.Tensor,
                         stream=None) -> None:
    _check(_lib.hc_encode_pack_batch(items, len(items), block_size, sub_block, _ptr(ws), ws.numel(), _ptr(err),
                                     _stream(stream)), "hc_encode_pack_batch")


def hc_decode_batch(items, block_size: int, sub_block: int, ws: torch.Tensor, err: torch.Tensor,
                    stream=None) -> None:
    _check(_lib.hc_decode_batch(items, len(items), block_size, sub_block, _ptr(ws), ws.numel(), _ptr(err),
                                _stream(stream)), "hc_decode_batch")


def hc_decode_batch_selfsync(items, block_size: int, ws: torch.Tensor, err: torch.Tensor, stream=None) -> None:
    """Every item's blocks decoded without the sub-block index (items' sub_idx unused)."""
    _check(_lib.hc_decode_batch_selfsync(items, len(items), block_size, _ptr(ws), ws.numel(), _ptr(err),
                                         _stream(stream)), "hc_decode_batch_selfsync")


def hc_probe_copy(src: torch.Tensor, dst: torch.Tensor, stream=None) -> None:
    """dst[:] = src[:] with the library's streaming copy probe (byte sizes equal, a multiple of 16)."""
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != n:
        raise ValueError("hc_probe_copy: src and dst differ in size")
    _check(_lib.hc_probe_copy(_ptr(src), _ptr(dst), n, _stream(stream)), "hc_probe_copy")


def hc_probe_read(src: torch.Tensor, sink: torch.Tensor, stream=None) -> None:
    """Reads all of src (a multiple of 16 bytes) and xors its 32-bit words into sink[0] (int32)."""
    n = src.numel() * src.element_size()
    _check(_lib.hc_probe_read(_ptr(src), n, _ptr(sink), _stream(stream)), "hc_probe_read")


def hc_copy(src: torch.Tensor, dst: torch.Tensor, stream=None) -> None:
    """dst[:] = src[:] by the library's copy kernel (device memory or pinned
    host memory on either side; byte sizes equal, a multiple of 16)."""
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != n:
        raise ValueError("hc_copy: src and dst differ in size")
    _check(_lib.hc_copy(_ptr(src), _ptr(dst), n, _stream(stream)), "hc_copy")
