"""Continuous-batching request loop over the batched codec calls.

Requests (compress a device buffer / decompress an encoded stream) arrive at
any time.  Every engine iteration, without waiting for work already on the
GPU:

  1. retires the batches whose completion event has fired: their requests
     get a completion time and their HBM reservation is released;
  2. admits waiting requests in arrival order while their device footprint
     fits the HBM budget: input, offsets and index (a decompress request:
     its stream and output); a compress request's output is reserved in a
     second stage, once its code and so its bound are known;
  3. launches one batch per phase over the newly admitted requests: block
     decode of the decompress requests (hc_decode_batch) on the decode
     stream; symbol counts of the compress requests (hc_histogram_batch) on
     the count stream, with an asynchronous 2 KiB-per-request copy of the
     counts to pinned host memory;
  4. for every compress batch whose counts have arrived (its event fired):
     builds the codes on the host, reserves the outputs (or waits, admitting
     nothing new meanwhile), takes resident code tables from the pool and
     launches the block encode (hc_encode_batch) on the encode stream,
     followed by an asynchronous copy of the batch's offset tables (whose
     last entries are the stream sizes) to pinned host memory.

The loop never blocks on the device: it only polls events, so requests that
arrive while others are on the GPU are admitted as soon as memory frees up,
and their kernels overlap the batches still running.  Code tables stay
resident on the device for the life of the request.  A result does not
depend on what it was batched with: the kernels treat every buffer as an
independent job (one table per job, offsets relative to its own stream).
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
               hc_sub_index_entries, make_items, new_error_word, num_blocks, set_item)

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


# The code length a compress request's output is first reserved for: its
# code is not known at admission.  Codes of the data served here stay well
# below it; a longer code takes the difference at its encode (see Server).
ESTIMATE_LEN = 16


def footprint(req: Request, block_size: int, sub_block: int) -> int:
    """Device bytes a request holds from admission: its input, and for a
    compress request its counts, offsets, sub-block index and an output
    sized for codes of ESTIMATE_LEN bits (corrected to its code's bound when
    the code is known); for a decompress request, its stream and output."""
    n = req.n
    nb = num_blocks(n, block_size)
    sub = 4 * hc_sub_index_entries(n, block_size, sub_block) if sub_block else 0
    if req.kind == "compress":
        return (_round(n) + _round(8 * (nb + 1)) + _round(sub) + 2048 +
                output_footprint(n, block_size, ESTIMATE_LEN))
    return _round(req.encoded.nbytes) + _round(max(n, 16))


def output_footprint(n: int, block_size: int, max_len: int) -> int:
    """Device bytes of a compress request's output buffer for codes of at most
    max_len bits (the second stage of its admission)."""
    return _round(max(hc_encode_bound(n, block_size, max_len), 16))


def worst_footprint(req: Request, block_size: int, sub_block: int) -> int:
    """The footprint with the longest possible codes: what a request may need
    at most, and so what must fit the budget for it to be admitted at all."""
    if req.kind != "compress":
        return footprint(req, block_size, sub_block)
    return (footprint(req, block_size, sub_block) - output_footprint(req.n, block_size, ESTIMATE_LEN) +
            output_footprint(req.n, block_size, 64))


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

    def submit(self, req, worst: Optional[int] = None) -> None:
        if (req.footprint if worst is None else worst) > self.budget:
            raise ValueError("request larger than the HBM budget")
        self.waiting.append(req)

    def admit(self, now: float, hold: bool = False) -> list:
        """Admits the head of the queue while it has arrived and fits; 'hold'
        admits nothing (a batch admitted earlier waits for its second stage)."""
        out = []
        while not hold and self.waiting and len(out) < self.max_batch:
            req = self.waiting[0]
            if req.arrival > now or self.in_use + req.footprint > self.budget:
                break
            self.waiting.popleft()
            self.in_use += req.footprint
            req.admitted = now
            out.append(req)
        return out

    def adjust(self, req, delta: int) -> bool:
        """Changes an admitted request's footprint by delta bytes (its output
        reservation corrected to its code): a decrease always, an increase
        only if it fits."""
        if delta > 0 and self.in_use + delta > self.budget:
            return False
        self.in_use += delta
        req.footprint += delta
        return True

    def release(self, req) -> None:
        self.in_use -= req.footprint
        assert self.in_use >= 0


@dataclass
class _Batch:
    requests: List[Request]
    event: torch.cuda.Event
    keep: list  # workspaces and item tables that must live until the batch ends
    errh: torch.Tensor  # pinned copy of the batch's error word
    offs: Optional[torch.Tensor] = None  # compress: pinned copy of the batch's offset tables
    last: Optional[List[int]] = None  # compress: index in offs of every request's stream size


@dataclass
class _Counting:
    """A compress batch whose symbol counts are on their way to the host, then
    (codes built) waiting for its outputs' reservation and code tables."""

    requests: List[Request]
    event: torch.cuda.Event
    hists: torch.Tensor  # pinned int64[count, 256]
    keep: list
    off_all: torch.Tensor  # the batch's offset tables, back to back
    last: List[int]  # index in off_all of every request's stream size
    codes: Optional[list] = None  # the requests' host codebooks, once the counts arrived
    out_delta: Optional[list] = None  # each output's bound minus what admission reserved for it


class Server:
    def __init__(self, block_size: int = 65536, sub_block: int = 128, hbm_budget: int = 32 << 30,
                 max_batch: int = 4096, device="cuda", clock=time.perf_counter, tables: int = 1024,
                 on_done=None):
        """on_done(request), if given, is called as each request retires (its
        result set); the server then keeps no list of finished requests."""
        self.B, self.S = block_size, sub_block
        self.on_done = on_done
        self.adm = Admission(hbm_budget, max_batch)
        self.device = torch.device(device)
        self.clock = clock
        self.inflight: List[_Batch] = []
        self.counting: List[_Counting] = []
        self.done: List[Request] = []
        self.hist_stream = torch.cuda.Stream(device=self.device)
        self.enc_stream = torch.cuda.Stream(device=self.device)
        self.dec_stream = torch.cuda.Stream(device=self.device)
        # Resident code tables, uploaded here: a compress request takes one
        # and refreshes it with an asynchronous copy, so no request waits for
        # a table allocation or a synchronous upload.  Results keep theirs
        # until handed back with recycle().  Only when every table is held by
        # results the caller has not recycled, with nothing in flight, does
        # the pool grow (an upload; counted in table_growths).
        self._one = np.zeros(256, np.uint8)
        self._one[0] = 1
        self._free_cb: List[DeviceCodebook] = [DeviceCodebook(hc_codebook_from_lengths(self._one))
                                               for _ in range(tables)]
        self._next_id = 0
        self.iterations = 0
        self.max_inflight_requests = 0
        self.table_growths = 0

    # ------------------------------------------------------------ queueing
    def submit(self, req: Request) -> Request:
        if req.kind not in ("compress", "decompress"):
            raise ValueError(req.kind)
        if req.kind == "decompress" and (req.encoded.block_size != self.B or req.encoded.sub_block != self.S):
            raise ValueError("decompress request encoded with another block size or index stride")
        req.rid = self._next_id
        self._next_id += 1
        req.footprint = footprint(req, self.B, self.S)
        self.adm.submit(req, worst_footprint(req, self.B, self.S))
        return req

    @property
    def waiting(self):
        return self.adm.waiting

    @property
    def in_use(self) -> int:
        return self.adm.in_use

    @property
    def idle(self) -> bool:
        """Nothing waiting, counting or on the device."""
        return not (self.waiting or self.counting or self.inflight)

    def _retire(self, now: float) -> int:
        still, retired = [], 0
        for b in self.inflight:
            if b.event.query():
                e = int(b.errh[0]) & 0xFFFFFFFF
                if e:
                    raise HcError(e, "batch (device)")
                offs = b.offs.numpy() if b.offs is not None else None
                for k, r in enumerate(b.requests):
                    if r.kind == "compress":
                        C = int(offs[b.last[k]])
                        # the result owns the tables it was encoded with (hand them back with recycle())
                        r.result = Encoded(r.bufs["out"][:C], r.bufs["off"], r.bufs["sub"], r.n, self.B, self.S,
                                           r.bufs["cb"])
                    else:
                        r.result = r.bufs["out"][: r.n]
                    r.completed = now
                    self.adm.release(r)
                    r.bufs = {}
                    if self.on_done is not None:
                        self.on_done(r)
                    else:
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
            errh = torch.empty(1, dtype=torch.int32, pin_memory=True)
            errh.copy_(err, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.dec_stream)
        self.inflight.append(_Batch(reqs, ev, [ws, items, err], errh))

    def _launch_counts(self, reqs: List[Request]):
        dev, B, S = self.device, self.B, self.S
        items = make_items(len(reqs))
        # the batch's counts, offset tables and index tables, each in one allocation
        nbs = [num_blocks(r.n, B) for r in reqs]
        subs = [max(hc_sub_index_entries(r.n, B, S), 1) for r in reqs] if S else None
        hist_all = torch.empty((len(reqs), 256), dtype=torch.int64, device=dev)
        off_all = torch.empty(sum(nbs) + len(reqs), dtype=torch.int64, device=dev)
        sub_all = torch.empty(sum(subs), dtype=torch.int32, device=dev) if S else None
        last, o, si = [], 0, 0
        for k, r in enumerate(reqs):
            r.bufs["hist"] = hist_all[k]
            r.bufs["off"] = off_all[o: o + nbs[k] + 1]
            last.append(o + nbs[k])
            o += nbs[k] + 1
            if S:
                r.bufs["sub"] = sub_all[si: si + subs[k]]
                si += subs[k]
            else:
                r.bufs["sub"] = None
            set_item(items, k, x=r.data, hist=r.bufs["hist"])
        self.hist_stream.wait_stream(torch.cuda.current_stream(dev))
        hists = torch.empty((len(reqs), 256), dtype=torch.int64, pin_memory=True)
        with torch.cuda.stream(self.hist_stream):
            hws = torch.empty(max(hc_batch_workspace_bytes(items, B), ALIGN), dtype=torch.uint8, device=dev)
            hc_histogram_batch(items, hws, stream=self.hist_stream)
            hists.copy_(hist_all, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.hist_stream)
        self.counting.append(_Counting(reqs, ev, hists, [hws, items], off_all, last))

    def _codes(self, c: _Counting):
        """The batch's codes from its counts (host), and its outputs' bytes."""
        hists = c.hists.numpy().view(np.uint64)
        c.codes = []
        for k, r in enumerate(c.requests):
            cb = hc_build_codebook(hists[k])
            if cb.max_len == 0:  # empty buffer: any one-symbol code
                cb = hc_codebook_from_lengths(self._one)
            c.codes.append(cb)
        c.out_delta = [output_footprint(r.n, self.B, cb.max_len) - output_footprint(r.n, self.B, ESTIMATE_LEN)
                       for r, cb in zip(c.requests, c.codes)]

    def _launch_encode(self, c: _Counting, m: int):
        """Encodes the batch's first m requests and drops them from it."""
        dev, B, S = self.device, self.B, self.S
        reqs, codes, last = c.requests[:m], c.codes[:m], c.last[:m]
        c.requests, c.codes, c.last, c.out_delta = c.requests[m:], c.codes[m:], c.last[m:], c.out_delta[m:]
        items = make_items(len(reqs))
        self.enc_stream.wait_stream(torch.cuda.current_stream(dev))
        self.enc_stream.wait_event(c.event)
        offs = torch.empty(c.off_all.numel(), dtype=torch.int64, pin_memory=True)
        with torch.cuda.stream(self.enc_stream):
            for k, r in enumerate(reqs):
                cb = codes[k]
                r.bufs["cb"] = self._free_cb.pop()
                r.bufs["cb"].update(cb, stream=self.enc_stream)
                r.bufs["out"] = torch.empty(output_footprint(r.n, B, cb.max_len), dtype=torch.uint8, device=dev)
                set_item(items, k, x=r.data, dcb=r.bufs["cb"], out=r.bufs["out"], block_off=r.bufs["off"],
                         sub_idx=r.bufs["sub"])
            ws = torch.empty(max(hc_batch_workspace_bytes(items, B), ALIGN), dtype=torch.uint8, device=dev)
            err = new_error_word(dev)
            hc_encode_batch(items, B, S, ws, err, stream=self.enc_stream)
            # every stream's size is its last offset: the batch's offset tables
            # (8 bytes per block) come back in one copy
            offs.copy_(c.off_all, non_blocking=True)
            errh = torch.empty(1, dtype=torch.int32, pin_memory=True)
            errh.copy_(err, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.enc_stream)
        self.inflight.append(_Batch(reqs, ev, c.keep + [ws, items, err], errh, offs, last))

    # ------------------------------------------------------------ the loop
    def step(self) -> int:
        """One engine iteration; returns the number of requests retired."""
        now = self.clock()
        retired = self._retire(now)
        # compress batches whose counts are here: codes on the host, each
        # output's reservation corrected to its code's bound, then the encode
        # of the longest prefix whose growth fits the budget and that has
        # free tables.  While part of a batch waits, nothing new is admitted;
        # the batches around it (whose reservations already cover them) go
        # ahead and free memory as they finish.
        still, hold = [], False
        for c in self.counting:
            if not c.event.query():
                still.append(c)
                continue
            if c.codes is None:
                self._codes(c)
                for r, d in zip(c.requests, c.out_delta):
                    if d < 0:
                        self.adm.adjust(r, d)  # the code is shorter than the estimate: give the rest back
            if len(self._free_cb) < len(c.requests) and not self.inflight:
                grow = len(c.requests) - len(self._free_cb)
                self._free_cb += [DeviceCodebook(hc_codebook_from_lengths(self._one)) for _ in range(grow)]
                self.table_growths += grow
            m = 0
            while m < min(len(c.requests), len(self._free_cb)):
                d = c.out_delta[m]
                if d > 0:
                    if not self.adm.adjust(c.requests[m], d):
                        break
                    c.out_delta[m] = 0  # reserved now
                m += 1
            if m:
                self._launch_encode(c, m)
            if c.requests:
                still.append(c)
                hold = True
        self.counting = still
        admitted = self.adm.admit(now, hold=hold)
        if admitted:
            self.iterations += 1
            deco = [r for r in admitted if r.kind == "decompress"]
            comp = [r for r in admitted if r.kind == "compress"]
            if deco:
                self._launch_decode(deco)
            if comp:
                self._launch_counts(comp)
        n_inflight = sum(len(b.requests) for b in self.inflight) + sum(len(c.requests) for c in self.counting)
        self.max_inflight_requests = max(self.max_inflight_requests, n_inflight)
        return retired

    def run_until_idle(self, stall_seconds: float = 60.0):
        """Steps until nothing is waiting, counting or on the device.  Raises
        if nothing retires, launches or arrives for stall_seconds (a budget
        too small for the requests in it)."""
        last = self.clock()
        while not self.idle:
            before = (len(self.waiting), len(self.counting), len(self.inflight))
            if self.step() or (len(self.waiting), len(self.counting), len(self.inflight)) != before:
                last = self.clock()
            elif self.clock() - last > stall_seconds:
                raise RuntimeError("serving loop made no progress (budget too small for the admitted requests)")
            if not self.inflight and not self.counting and self.waiting:
                # idle until the next arrival: sleep only to within 0.5 ms of
                # it and poll from there, so that an oversleeping timer never
                # adds to a request's latency (an iteration with nothing on
                # the device is cheap)
                wait = self.waiting[0].arrival - self.clock()
                if wait > 0.001:
                    time.sleep(min(wait - 0.0005, 0.002))
                if wait > 0:
                    last = self.clock()
        return self.done


def percentile(values, q: float) -> float:
    return float(np.percentile(np.asarray(values, dtype=np.float64), q)) if len(values) else float("nan")
