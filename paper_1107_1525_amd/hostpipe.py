"""Host-resident data through the device coder, with the transfers overlapped.

The paper's conclusion (section 4) finds the GPU coder weighed down by
moving data between host and device, and proposes overlapping the transfers
with the coding.  Here a pinned host buffer is cut into chunks of M bytes (M a
multiple of the block size B; the last chunk may be short).  Each chunk is
one independent stream with its own code, built from its own symbol counts
(section 2 counts the symbols of each stream), and three HIP streams overlap:

  copy-in   chunk k+1, k+2  host -> device (PCIe, one direction); when
                            decompressing, the chunk's code tables too
  coding    chunk k         counts, code tables and block encode; or decode
  copy-out  chunk k-1       device -> host (PCIe, the other direction)

Device buffers form a ring of `slots` chunk slots; events order each slot's
reuse (its copy-in waits until the coding of the chunk that last held it has
read it, its coding waits until that chunk's copy-out has drained it).

When decompressing, copies out go through the library's copy kernel
(hc_copy: one work-group per CU, straight into the pinned buffer): the
runtime sent some 64 MiB device-to-host copies to an SDMA engine at about a
quarter of its blit kernel's rate.  When compressing, the runtime copies out
(there the copy kernel's groups took CU slots from the encode kernels and
the runtime did better); copies in stay with the runtime.

Compressing needs two host waits per chunk: the chunk's 2 KiB of counts (the
code is built on the host) and its compressed size (the copy-out moves
exactly C_k bytes).  Decompressing has none: sizes and codes are known.

All arithmetic runs in the library's kernels; this module only orders copies
and launches.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from . import (DeviceCodebook, HcError, HC_ERR_NO_SPACE, hc_build_codebook, hc_codebook_from_lengths, hc_copy,
               hc_decode_blocks, hc_encode_blocks, hc_encode_bound, hc_encode_workspace_bytes, hc_histogram,
               hc_sub_index_entries, num_blocks, read_error)


def plan_chunks(n: int, chunk_bytes: int, block_size: int) -> List[tuple]:
    """[(start, length)] of the chunks of an n-byte buffer: whole chunks of
    chunk_bytes, the last one short.  chunk_bytes must be a positive multiple
    of block_size, so that a chunk's blocks are the buffer's blocks."""
    if block_size <= 0 or chunk_bytes <= 0 or chunk_bytes % block_size:
        raise ValueError("chunk_bytes must be a positive multiple of block_size")
    return [(a, min(chunk_bytes, n - a)) for a in range(0, n, chunk_bytes)]


@dataclass
class HostChunk:
    """One chunk of a host-resident encoding: its stream occupies
    data[pos : pos + nbytes] (pos a multiple of 16); lengths (256 u8) determine its canonical code;
    block_off (nb + 1 u64 as int64) and sub_idx (int32, or None) are pinned
    host tensors."""
    start: int
    n: int
    pos: int
    nbytes: int
    lengths: np.ndarray
    block_off: torch.Tensor
    sub_idx: Optional[torch.Tensor]


@dataclass
class HostEncoded:
    data: torch.Tensor  # pinned uint8: the chunks' streams in order, each from a 16-byte boundary
    total: int
    n: int
    block_size: int
    sub_block: int
    chunk_bytes: int
    chunks: List[HostChunk] = field(default_factory=list)


class HostPipeline:
    """Compress and decompress pinned host buffers on one device, chunk by
    chunk, with copy-in, coding and copy-out overlapped on three streams."""

    def __init__(self, block_size: int, sub_block: int = 0, chunk_bytes: int = 64 << 20, slots: int = 3,
                 device: int = 0):
        if slots < 2:
            raise ValueError("slots must be >= 2")
        plan_chunks(chunk_bytes, chunk_bytes, block_size)  # validates the sizes
        self.B, self.S, self.M, self.slots = block_size, sub_block, chunk_bytes, slots
        self.dev = torch.device("cuda", device)
        self.s_in = torch.cuda.Stream(self.dev)
        self.s_code = torch.cuda.Stream(self.dev)
        self.s_out = torch.cuda.Stream(self.dev)
        M, B, S = self.M, self.B, self.S
        nb = num_blocks(M, B)
        u8 = dict(dtype=torch.uint8, device=self.dev)
        self.d_x = [torch.empty(M, **u8) for _ in range(slots)]
        self.d_cap = [0] * slots
        self.d_z = [torch.empty(16, **u8) for _ in range(slots)]  # streams: grown to the code's bound
        self.d_off = [torch.empty(nb + 1, dtype=torch.int64, device=self.dev) for _ in range(slots)]
        self.d_sub = [torch.empty(max(hc_sub_index_entries(M, B, S), 1), dtype=torch.int32, device=self.dev)
                      if S else None for _ in range(slots)]
        self.d_hist = [torch.empty(256, dtype=torch.int64, device=self.dev) for _ in range(slots)]
        self.h_hist = [torch.empty(256, dtype=torch.int64).pin_memory() for _ in range(slots)]
        self.ws = [torch.empty(max(hc_encode_workspace_bytes(M, B), 16), **u8) for _ in range(slots)]
        self.err = torch.zeros(1, dtype=torch.int32, device=self.dev)
        L = np.zeros(256, np.uint8)
        L[0] = 1
        # code tables: compressing refreshes slot k % slots on the coding
        # stream; decompressing refreshes handle k % (2 slots) on the copy-in
        # stream, so that the host-side wait of a refresh (for the handle's
        # previous table copy) is on a copy two rounds of slots back
        self.dcb = [DeviceCodebook(hc_codebook_from_lengths(L)) for _ in range(2 * slots)]
        self.kernel_copy = True  # until the runtime says a buffer is not device-visible

    def _copy_out(self, src: torch.Tensor, dst: torch.Tensor):
        """src (device) into dst (pinned host) on the copy-out stream: the
        library's copy kernel for the 16-byte-multiple head when both ends are
        16-byte aligned, the runtime for the rest."""
        n = src.numel()
        head = n - n % 16
        if not (self.kernel_copy and head and src.data_ptr() % 16 == 0 and dst.data_ptr() % 16 == 0):
            head = 0
        if head:
            try:
                hc_copy(src[:head], dst[:head], stream=self.s_out)
            except HcError:
                self.kernel_copy = False  # not device-visible at its own address: the runtime copies
                head = 0
        if head < n:
            dst[head:].copy_(src[head:], non_blocking=True)

    def _drain(self):
        for st in (self.s_in, self.s_code, self.s_out):
            st.synchronize()

    def _ensure_out(self, slot: int, cap: int, free_ev):
        if self.d_cap[slot] >= cap:
            return
        if free_ev is not None:
            free_ev.synchronize()  # the slot's last copy-out has drained it
        self.d_z[slot] = torch.empty((cap + 255) // 256 * 256, dtype=torch.uint8, device=self.dev)
        self.d_cap[slot] = self.d_z[slot].numel()

    def compress(self, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> HostEncoded:
        """x: pinned uint8 host tensor.  out: optional pinned uint8 host tensor
        for the streams (by default sized for codes of up to 8 bits, n plus
        the headers and pads; a larger code raises HcError NO_SPACE if the
        streams do not fit)."""
        assert x.dtype == torch.uint8 and not x.is_cuda and x.is_contiguous()
        n, B, S, K = x.numel(), self.B, self.S, self.slots
        plan = plan_chunks(n, self.M, B)
        if out is None:
            out = torch.empty(max(sum(hc_encode_bound(m, B, 8) + 16 for _, m in plan), 16),
                              dtype=torch.uint8).pin_memory()
        nbs = [num_blocks(m, B) for _, m in plan]
        off_h = torch.empty(sum(nb + 1 for nb in nbs) or 1, dtype=torch.int64).pin_memory()
        nsub = [hc_sub_index_entries(m, B, S) if S else 0 for _, m in plan]
        sub_h = torch.empty(max(sum(nsub), 1), dtype=torch.int32).pin_memory() if S else None
        enc = HostEncoded(out, 0, n, B, S, self.M)
        ev_in, ev_hist, ev_enc, ev_out = {}, {}, {}, {}
        self.err.zero_()
        torch.cuda.current_stream(self.dev).synchronize()

        def issue_in(j):
            slot = j % K
            a, m = plan[j]
            with torch.cuda.stream(self.s_in):
                if j - K in ev_enc:
                    self.s_in.wait_event(ev_enc[j - K])  # the slot's last coding has read it
                self.d_x[slot][:m].copy_(x[a:a + m], non_blocking=True)
                ev_in[j] = torch.cuda.Event()
                ev_in[j].record(self.s_in)

        def issue_counts(j):
            slot = j % K
            m = plan[j][1]
            with torch.cuda.stream(self.s_code):
                self.s_code.wait_event(ev_in[j])
                hc_histogram(self.d_x[slot][:m], self.d_hist[slot], stream=self.s_code)
                self.h_hist[slot].copy_(self.d_hist[slot], non_blocking=True)
                ev_hist[j] = torch.cuda.Event()
                ev_hist[j].record(self.s_code)

        obase = np.cumsum([0] + [nb + 1 for nb in nbs])
        sbase = np.cumsum([0] + nsub)
        pos = 0

        def issue_out(j):
            nonlocal pos
            slot = j % K
            a, m = plan[j]
            ev_enc[j].synchronize()  # the chunk's offsets are on the host
            offs = off_h[obase[j]:obase[j + 1]]
            C = int(offs[nbs[j]])
            pos = (pos + 15) // 16 * 16  # each chunk's stream from a 16-byte boundary
            if pos + C > out.numel():
                self._drain()  # nothing left in flight on the caller's buffers
                raise HcError(HC_ERR_NO_SPACE, "HostPipeline.compress: output buffer too small")
            with torch.cuda.stream(self.s_out):
                self.s_out.wait_event(ev_enc[j])
                out[pos:pos + C].copy_(self.d_z[slot][:C], non_blocking=True)
                ev_out[j] = torch.cuda.Event()
                ev_out[j].record(self.s_out)
            enc.chunks[j].pos, enc.chunks[j].nbytes = pos, C
            pos += C

        nxt = 0
        for k, (a, m) in enumerate(plan):
            while nxt < len(plan) and nxt < k + K:
                issue_in(nxt)
                nxt += 1
            slot = k % K
            issue_counts(k)
            ev_hist[k].synchronize()
            cb = hc_build_codebook(self.h_hist[slot].numpy().view(np.uint64))
            self._ensure_out(slot, hc_encode_bound(m, B, int(cb.max_len)), ev_out.get(k - K))
            with torch.cuda.stream(self.s_code):
                if k - K in ev_out:
                    self.s_code.wait_event(ev_out[k - K])  # the slot's stream buffer has been copied out
                self.dcb[slot].update(cb, stream=self.s_code)
                hc_encode_blocks(self.d_x[slot][:m], B, self.dcb[slot], self.d_z[slot], self.d_off[slot][:nbs[k] + 1],
                                 self.d_sub[slot][:max(nsub[k], 1)] if S else None, S, self.ws[slot], self.err,
                                 stream=self.s_code)
                off_h[obase[k]:obase[k + 1]].copy_(self.d_off[slot][:nbs[k] + 1], non_blocking=True)
                if S:
                    sub_h[sbase[k]:sbase[k + 1]].copy_(self.d_sub[slot][:nsub[k]], non_blocking=True)
                ev_enc[k] = torch.cuda.Event()
                ev_enc[k].record(self.s_code)
            enc.chunks.append(HostChunk(a, m, 0, 0, np.array(cb.len[:], dtype=np.uint8),
                                        off_h[obase[k]:obase[k + 1]],
                                        sub_h[sbase[k]:sbase[k + 1]] if S else None))
            if k >= 1:
                issue_out(k - 1)
        if plan:
            issue_out(len(plan) - 1)
        self._drain()
        e = read_error(self.err)
        if e:
            raise HcError(e, "HostPipeline.compress (device)")
        enc.total = pos
        return enc

    def decompress(self, enc: HostEncoded, y: Optional[torch.Tensor] = None) -> torch.Tensor:
        """The encoding's bytes into a pinned uint8 host tensor of enc.n bytes."""
        if enc.block_size != self.B or enc.sub_block != self.S or enc.chunk_bytes > self.M:
            raise ValueError("HostPipeline.decompress: block size, sub-block or chunk size differ")
        if y is None:
            y = torch.empty(max(enc.n, 16), dtype=torch.uint8).pin_memory()[:enc.n]
        B, S, K = self.B, self.S, self.slots
        ev_in, ev_dec, ev_out = {}, {}, {}
        self.err.zero_()
        torch.cuda.current_stream(self.dev).synchronize()
        for k, c in enumerate(enc.chunks):
            slot = k % K
            nb = num_blocks(c.n, B)
            self._ensure_out(slot, c.nbytes, ev_dec.get(k - K))
            with torch.cuda.stream(self.s_in):
                if k - K in ev_dec:
                    self.s_in.wait_event(ev_dec[k - K])  # the slot's last decode has read its inputs and tables
                self.d_z[slot][:c.nbytes].copy_(enc.data[c.pos:c.pos + c.nbytes], non_blocking=True)
                self.d_off[slot][:nb + 1].copy_(c.block_off, non_blocking=True)
                if S:
                    self.d_sub[slot][:c.sub_idx.numel()].copy_(c.sub_idx, non_blocking=True)
                # the slot's code tables travel with its data: on the coding
                # stream their copy would queue behind the chunk copies
                self.dcb[k % (2 * K)].update(hc_codebook_from_lengths(c.lengths), stream=self.s_in)
                ev_in[k] = torch.cuda.Event()
                ev_in[k].record(self.s_in)
            with torch.cuda.stream(self.s_code):
                self.s_code.wait_event(ev_in[k])
                if k - K in ev_out:
                    self.s_code.wait_event(ev_out[k - K])  # the slot's output has been copied out
                hc_decode_blocks(self.d_z[slot], c.nbytes, c.n, B, self.dcb[k % (2 * K)], self.d_off[slot][:nb + 1],
                                 self.d_sub[slot] if S else None, S, self.d_x[slot][:c.n], self.err,
                                 stream=self.s_code)
                ev_dec[k] = torch.cuda.Event()
                ev_dec[k].record(self.s_code)
            with torch.cuda.stream(self.s_out):
                self.s_out.wait_event(ev_dec[k])
                self._copy_out(self.d_x[slot][:c.n], y[c.start:c.start + c.n])
                ev_out[k] = torch.cuda.Event()
                ev_out[k].record(self.s_out)
        self._drain()
        e = read_error(self.err)
        if e:
            raise HcError(e, "HostPipeline.decompress (device)")
        return y
