"""Continuous-batching request loop over the batched codec calls.

Requests (compress a device buffer / decompress an encoded stream) arrive at
any time.  Every engine iteration, without waiting for work already on the
GPU:

  1. retires the batches whose completion event has fired: their requests
     get a completion time and their HBM reservation is released;
  2. admits waiting requests in arrival order while their device footprint
     (input + output + offsets + index) fits the HBM budget;
  3. launches one batch per phase over the newly admitted requests: block
     decode of the decompress requests (hc_decode_batch) on the decode
     stream; symbol counts of the compress requests (hc_histogram_batch),
     the 2 KiB-per-request read-back, the host code build, and their block
     encode (hc_encode_batch) on the encode stream.

So requests that arrive while others are on the GPU are admitted as soon as
memory frees up, and their kernels overlap the batches still running.  Code
tables stay resident on the device for the life of the request.  A result
does not depend on what it was batched with: the kernels treat every buffer
as an independent job (one table per job, offsets relative to its own
stream).
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import Deque, List, Optional

import numpy as np
import torch

from . import (DeviceCodebook, Encoded, HcError, hc_batch_workspace_bytes, hc_build_codebook,
               hc_codebook_from_lengths, hc_decode_batch, hc_encode_batch, hc_encode_bound, hc_histogram_batch,
               hc_sub_index_entries, make_items, new_error_word, num_blocks, read_error, set_item)

ALIGN = 256


def _round(x: int) -> int:
    return (x + ALIGN - 1) // ALIGN * ALIGN


@dataclass
class Request:
    """A compress request carries `data` (uint8 device tensor); a decompress
    request carries `encoded`.  Times are seconds on the server's clock."""

    kind: str  # "compress" or "decompress"
    data: Optional[torch.Tensor] = None
    encoded: Optional[Encoded] = None
    arrival: float = 0.0
    rid: int = 0
    admitted: Optional[float] = None
    completed: Optional[float] = None
    result: object = None
    footprint: int = 0
    bufs: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.data.numel() if self.kind == "compress" else self.encoded.n

    @property
    def latency(self) -> Optional[float]:
        return None if self.completed is None else self.completed - self.arrival


def footprint(req: Request, block_size: int, sub_block: int) -> int:
    """Device bytes a request holds while in flight: its input, the output the
    server allocates for it (sized for 64-bit codes before the code is known),
    offsets and sub-block index."""
    n = req.n
    nb = num_blocks(n, block_size)
    sub = 4 * hc_sub_index_entries(n, block_size, sub_block) if sub_block else 0
    if req.kind == "compress":
        return _round(n) + _round(hc_encode_bound(n, block_size, 64)) + _round(8 * (nb + 1)) + _round(sub) + 2048
    return _round(req.encoded.nbytes) + _round(max(n, 16))


class Admission:
    """FIFO admission by device footprint: the head of the queue is admitted
    once it has arrived and its footprint fits what is left of the budget;
    nothing behind it is admitted first, so no request starves.  Pure host
    logic (no GPU), shared by the server and its CPU tests."""

    def __init__(self, budget: int, max_batch: int = 1 << 30):
        self.budget = budget
        self.max_batch = max_batch
        self.waiting: Deque = deque()
        self.in_use = 0

    def submit(self, req) -> None:
        if req.footprint > self.budget:
            raise ValueError("request larger than the HBM budget")
        self.waiting.append(req)

    def admit(self, now: float) -> list:
        out = []
        while self.waiting and len(out) < self.max_batch:
            req = self.waiting[0]
            if req.arrival > now or self.in_use + req.footprint > self.budget:
                break
            self.waiting.popleft()
            self.in_use += req.footprint
            req.admitted = now
            out.append(req)
        return out

    def release(self, req) -> None:
        self.in_use -= req.footprint
        assert self.in_use >= 0


@dataclass
class _Batch:
    requests: List[Request]
    event: torch.cuda.Event
    keep: list  # workspaces and item tables that must live until the batch ends
    err: torch.Tensor


class Server:
    def __init__(self, block_size: int = 65536, sub_block: int = 1024, hbm_budget: int = 32 << 30,
                 max_batch: int = 4096, device="cuda", clock=time.perf_counter):
        self.B, self.S = block_size, sub_block
        self.adm = Admission(hbm_budget, max_batch)
        self.device = torch.device(device)
        self.clock = clock
        self.inflight: List[_Batch] = []
        self.done: List[Request] = []
        self.hist_stream = torch.cuda.Stream(device=self.device)
        self.enc_stream = torch.cuda.Stream(device=self.device)
        self.dec_stream = torch.cuda.Stream(device=self.device)
        self._free_cb: List[DeviceCodebook] = []  # resident code tables handed back by recycle()
        self._next_id = 0
        self.iterations = 0
        self.max_inflight_requests = 0

    # ------------------------------------------------------------ queueing
    def submit(self, req: Request) -> Request:
        if req.kind not in ("compress", "decompress"):
            raise ValueError(req.kind)
        if req.kind == "decompress" and (req.encoded.block_size != self.B or req.encoded.sub_block != self.S):
            raise ValueError("decompress request encoded with another block size or index stride")
        req.rid = self._next_id
        self._next_id += 1
        req.footprint = footprint(req, self.B, self.S)
        self.adm.submit(req)
        return req

    @property
    def waiting(self):
        return self.adm.waiting

    @property
    def in_use(self) -> int:
        return self.adm.in_use

    def _retire(self, now: float) -> int:
        still, retired = [], 0
        for b in self.inflight:
            if b.event.query():
                e = read_error(b.err)
                if e:
                    raise HcError(e, "batch (device)")
                for r in b.requests:
                    if r.kind == "compress":
                        nb = num_blocks(r.n, self.B)
                        C = int(r.bufs["off"][nb].item())
                        # the result owns the tables it was encoded with (hand them back with recycle())
                        r.result = Encoded(r.bufs["out"][:C], r.bufs["off"], r.bufs["sub"], r.n, self.B, self.S,
                                           r.bufs["cb"])
                    else:
                        r.result = r.bufs["out"][: r.n]
                    r.completed = now
                    self.adm.release(r)
                    r.bufs = {}
                    self.done.append(r)
                    retired += 1
            else:
                still.append(b)
        self.inflight = still
        return retired

    def recycle(self, encoded: Encoded):
        """Returns the device code tables of a compress result that is no
        longer needed; later requests reuse them (refreshed asynchronously)."""
        if encoded.codebook is not None:
            self._free_cb.append(encoded.codebook)
            encoded.codebook = None

    # ------------------------------------------------------------ launches
    def _launch_decode(self, reqs: List[Request]):
        dev = self.device
        items = make_items(len(reqs))
        for k, r in enumerate(reqs):
            e = r.encoded
            r.bufs["out"] = torch.empty(max(r.n, 16), dtype=torch.uint8, device=dev)
            set_item(items, k, x=e.stream, n=e.n, in_bytes=e.nbytes, dcb=e.codebook, out=r.bufs["out"],
                     block_off=e.block_off, sub_idx=e.sub_idx)
        self.dec_stream.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(self.dec_stream):
            ws = torch.empty(max(hc_batch_workspace_bytes(items, self.B), ALIGN), dtype=torch.uint8, device=dev)
            err = new_error_word(dev)
            hc_decode_batch(items, self.B, self.S, ws, err, stream=self.dec_stream)
            ev = torch.cuda.Event()
            ev.record(self.dec_stream)
        self.inflight.append(_Batch(reqs, ev, [ws, items], err))

    def _launch_compress(self, reqs: List[Request]):
        dev, B, S = self.device, self.B, self.S
        items = make_items(len(reqs))
        for k, r in enumerate(reqs):
            r.bufs["hist"] = torch.empty(256, dtype=torch.int64, device=dev)
            r.bufs["off"] = torch.empty(num_blocks(r.n, B) + 1, dtype=torch.int64, device=dev)
            r.bufs["sub"] = (torch.empty(max(hc_sub_index_entries(r.n, B, S), 1), dtype=torch.int32, device=dev)
                             if S else None)
            set_item(items, k, x=r.data, hist=r.bufs["hist"])
        main = torch.cuda.current_stream(dev)
        self.hist_stream.wait_stream(main)
        with torch.cuda.stream(self.hist_stream):
            hws = torch.empty(max(hc_batch_workspace_bytes(items, B), ALIGN), dtype=torch.uint8, device=dev)
            hc_histogram_batch(items, hws, stream=self.hist_stream)
            # the read-back waits for the counting only, not for batches on the other streams
            hists = torch.stack([r.bufs["hist"] for r in reqs]).cpu().numpy().view(np.uint64)
        self.enc_stream.wait_stream(main)
        with torch.cuda.stream(self.enc_stream):
            for k, r in enumerate(reqs):
                cb = hc_build_codebook(hists[k])
                if cb.max_len == 0:  # empty buffer: any one-symbol code
                    L = np.zeros(256, np.uint8)
                    L[0] = 1
                    cb = hc_codebook_from_lengths(L)
                if self._free_cb:
                    r.bufs["cb"] = self._free_cb.pop()
                    r.bufs["cb"].update(cb, stream=self.enc_stream)
                else:
                    r.bufs["cb"] = DeviceCodebook(cb)
                r.bufs["out"] = torch.empty(_round(max(hc_encode_bound(r.n, B, cb.max_len), 16)), dtype=torch.uint8,
                                            device=dev)
                set_item(items, k, x=r.data, dcb=r.bufs["cb"], out=r.bufs["out"], block_off=r.bufs["off"],
                         sub_idx=r.bufs["sub"])
            ws = torch.empty(max(hc_batch_workspace_bytes(items, B), ALIGN), dtype=torch.uint8, device=dev)
            err = new_error_word(dev)
            hc_encode_batch(items, B, S, ws, err, stream=self.enc_stream)
            ev = torch.cuda.Event()
            ev.record(self.enc_stream)
        self.inflight.append(_Batch(reqs, ev, [hws, ws, items], err))

    # ------------------------------------------------------------ the loop
    def step(self) -> int:
        """One engine iteration; returns the number of requests retired."""
        now = self.clock()
        retired = self._retire(now)
        admitted = self.adm.admit(now)
        if admitted:
            self.iterations += 1
            deco = [r for r in admitted if r.kind == "decompress"]
            comp = [r for r in admitted if r.kind == "compress"]
            if deco:
                self._launch_decode(deco)
            if comp:
                self._launch_compress(comp)
        n_inflight = sum(len(b.requests) for b in self.inflight)
        self.max_inflight_requests = max(self.max_inflight_requests, n_inflight)
        return retired

    def run_until_idle(self):
        while self.waiting or self.inflight:
            self.step()
            if not self.inflight and self.waiting:
                wait = self.waiting[0].arrival - self.clock()
                if wait > 0:
                    time.sleep(min(wait, 0.002))
        return self.done


def percentile(values, q: float) -> float:
    return float(np.percentile(np.asarray(values, dtype=np.float64), q)) if len(values) else float("nan")
