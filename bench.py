"""Benchmark of the block-decomposed Huffman codec on one MI355X.

One step = the whole coding path over the 4 GiB mixed workload (64 segments of
64 MiB cycling uniform / skewed / fp32 bytes, one codebook per segment):

  1. symbol counts of every segment            (hc_histogram_batch, one launch)
  2. read-back of the 64 histograms (16 KiB)
  3. Huffman code + canonical codes of every segment and one refresh of the
     resident device tables                     (hc_cbset_build, host + async copy)
  4. block encode of every segment: length pass, offset scan, bit packing
                                                (hc_encode_batch, one launch each)
  5. block decode of every segment from the encoder's offsets and sub-block
     index                                      (hc_decode_batch: one launch for
                                                the complete 8-bit codes, one
                                                for the rest)

Steps are pipelined: step k+1's counts are launched before step k's decode,
so the host builds step k+1's codes while the device decodes step k.

Inputs are resident in HBM before timing starts.  The JSON line reports the
whole-step throughput in uncompressed GB/s, the per-phase rates, the roofline
of the dominant kernel (its algorithmic bytes per launch over its average
launch time, timed with HIP events on the stream it runs on), and the CPU
oracle timed on a bounded sample of the same workload.

  python bench.py [--steps K] [--warmup W] [--block B] [--sub-block S]
  python bench.py --sweep          # block size / sub-block sweep, one line each
  python bench.py --copy-probe     # streaming copy / read probes: achievable HBM GB/s
  python bench.py --batched N      # + N independent buffers, batched / graph / plain
  python bench.py --serve N        # + the serving loop against one request per launch
  python bench.py --host-pipeline  # + the workload from pinned host memory, PCIe included
  python bench.py --no-selfsync    # without the decodes that use no sub-block index
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, vendor figure
METRIC = "compress/decompress GB/s (uncompressed) and % HBM peak; batched p50/p99 latency"
WORKLOAD = "mixed-4GiB-64x64MiB"
# the device function each timed launch runs (rocprofv3 names)
# the device function of each single launch the bench times (its rocprofv3
# name without template arguments); the packing has one instance per class
# in every call (the copy and the packing proper), so its traffic summary
# (instances summed per call) is not that of one launch
KERNEL_SYMBOL = {"k_hist": "k_hist", "k_count": "k_count", "k_offsets": "k_offsets", "k_encode": "k_encode",
                 "k_encode_copy": "k_encode", "k_encode_pack": "k_encode", "k_decode": "k_decode_stage",
                 "k_decode_copy": "k_decode_ring", "k_decode_table": "k_decode_stage"}
SINGLE_INSTANCE = ("k_hist", "k_count", "k_decode_copy", "k_decode_table")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--block", type=int, default=None,
                    help="block size B (default: the autotuner's choice among 4/16/64/256 KiB)")
    ap.add_argument("--sub-block", type=int, default=None,
                    help="sub-block index stride S (default: the autotuner's choice)")
    ap.add_argument("--tile-loads", type=int, default=None,
                    help="encode tile loads per thread, 0 (the library's rule), 1, 2 or 4 (default: autotuned)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner: B = 64 KiB, S = 128, the library's tile rule unless given")
    ap.add_argument("--tune-segments", type=int, default=12,
                    help="64 MiB segments of the mixed workload the autotuner measures on (default 12)")
    ap.add_argument("--segments", type=int, default=64, help="number of 64 MiB segments (64 = 4 GiB)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-step", action="store_true",
                    help="the timed step, its per-kernel and per-launch times and the probes only (no per-kind "
                         "split, single streams, batches, serving, index-free decodes or CPU baseline): the "
                         "command the kernel-trace and counter profiles run")
    ap.add_argument("--sweep", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--per-kind", action="store_true",
                    help="the same step on segments of one data kind at a time (uniform, skewed, fp32): "
                         "per-kernel time and GB/s of each kind, one JSON line each")
    ap.add_argument("--batched", type=int, default=10000, metavar="N",
                    help="N independent buffers (log-uniform 1 KiB-64 MiB, Zipf s in [0.8,1.6]): one launch per "
                         "phase, its graph replay, and one buffer per launch (0: skip)")
    ap.add_argument("--serve", type=int, default=5500, metavar="N",
                    help="the serving loop on N requests (the first 500 warm-up; 50/50 compress/decompress, log-uniform "
                         "4 KiB-256 MiB, mixed data) against one request per launch: saturation GB/s of both, "
                         "and p50/p99 latency of both under the same Poisson arrivals at 0.5 and 0.8 load (0: skip)")
    ap.add_argument("--host-pipeline", action="store_true",
                    help="also run the workload from pinned host memory through the chunked pipeline "
                         "(copy-in, coding, copy-out overlapped; 64 MiB chunks, one code each): "
                         "PCIe-inclusive compress / decompress GB/s beside plain pinned copy rates")
    ap.add_argument("--no-selfsync", action="store_true",
                    help="skip the decodes of the workload's streams without their sub-block index "
                         "(batched piece decoder and batched lane-per-block decode, beside the indexed one)")
    ap.add_argument("--traffic-summary", metavar="DIR",
                    help="turn rocprofv3 --pmc runs in DIR/{fetch,write,copy_fetch,copy_write} into "
                         "profiles/traffic_*.json (HBM bytes per launch of each codec kernel)")
    ap.add_argument("--trace-summary", metavar="DIR",
                    help="print the codec kernels' durations from a rocprofv3 --kernel-trace run of --only-step "
                         "(all dispatches, and those no other codec kernel overlapped)")
    ap.add_argument("--sq-table", metavar="DIR",
                    help="turn rocprofv3 --pmc runs of --per-kind under DIR (any number of counter sets) into "
                         "a per-kind table of SQ counters per symbol and per wave cycle of each codec kernel")
    return ap.parse_args()


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("hc_kernels.hip", "hc_kernels.h"):
        with open(os.path.join(ROOT, "paper_1107_1525_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


class Workload:
    """The 4 GiB mixed buffer and every device buffer one step needs.

    Each phase is one batched launch over all segments (hc_histogram_batch,
    hc_encode_batch, hc_decode_batch); the segment table lives in hc_item
    arrays built once."""

    def __init__(self, hc, synth, torch, nseg, B, S, kind=None):
        self.hc, self.torch = hc, torch
        self.seg = synth.WORKLOADS[WORKLOAD]["segment"]
        self.nseg = nseg
        self.n = self.seg * nseg
        self.B, self.S = B, S
        dev = "cuda"
        self.x = torch.empty(self.n, dtype=torch.uint8, device=dev)
        for t in range(nseg):
            synth.segment_bytes_torch(kind or synth.mixed_kind(t), self.seg, synth.derive_seed(3, t),
                                      out=self.x[t * self.seg:(t + 1) * self.seg])
        self.hist = torch.zeros((nseg, 256), dtype=torch.int64, device=dev)
        self.hist_host = torch.zeros((nseg, 256), dtype=torch.int64).pin_memory()
        self.hist_items = hc.make_items(nseg)
        for t in range(nseg):
            hc.set_item(self.hist_items, t, x=self.xs(t), hist=self.hist[t])
        self.hist_ws = torch.empty(max(hc.hc_batch_workspace_bytes(self.hist_items, B), 256),
                                   dtype=torch.uint8, device=dev)
        # codebooks of the data (fixed across steps) size the output buffers
        hc.hc_histogram_batch(self.hist_items, self.hist_ws)
        h = self.hist.cpu().numpy().view("uint64")
        self.cbset = hc.CodebookSet(nseg)  # resident tables, rebuilt every step
        self.dcb = self.cbset.build(h)
        self.nb = hc.num_blocks(self.seg, B)
        self.cap = [(hc.hc_encode_bound(self.seg, B, d.max_len) + 255) // 256 * 256 for d in self.dcb]
        self.out_base = [0]
        for c in self.cap:
            self.out_base.append(self.out_base[-1] + c)
        self.out = torch.empty(self.out_base[-1], dtype=torch.uint8, device=dev)
        self.off = torch.empty((nseg, self.nb + 1), dtype=torch.int64, device=dev)
        self.nsub = hc.hc_sub_index_entries(self.seg, B, S) if S else 0
        self.sub = torch.empty((nseg, max(self.nsub, 1)), dtype=torch.int32, device=dev) if S else None
        self.y = torch.empty(self.n, dtype=torch.uint8, device=dev)
        self.err = torch.zeros(1, dtype=torch.int32, device=dev)
        self.enc_items = hc.make_items(nseg)
        for t in range(nseg):
            hc.set_item(self.enc_items, t, x=self.xs(t), dcb=self.dcb[t], out=self.outs(t), block_off=self.off[t],
                        sub_idx=self.subs(t))
        self.ws = torch.empty(hc.hc_batch_workspace_bytes(self.enc_items, B), dtype=torch.uint8, device=dev)
        hc.hc_encode_batch(self.enc_items, B, S, self.ws, self.err)
        self.C = [int(v) for v in self.off[:, self.nb].cpu()]
        self.dec_items = hc.make_items(nseg)
        for t in range(nseg):
            hc.set_item(self.dec_items, t, x=self.outs(t), n=self.seg, in_bytes=self.C[t], dcb=self.dcb[t],
                        out=self.ys(t), block_off=self.off[t], sub_idx=self.subs(t))

    def xs(self, t):
        return self.x[t * self.seg:(t + 1) * self.seg]

    def ys(self, t):
        return self.y[t * self.seg:(t + 1) * self.seg]

    def outs(self, t):
        return self.out[self.out_base[t]:self.out_base[t] + self.cap[t]]

    def subs(self, t):
        return self.sub[t] if self.S else None

    def run(self, steps, evs=None):
        """'steps' passes of the whole path (one pass: counts, their read-back,
        host code build and one table copy, encode, decode), pipelined across
        passes: the counts of pass k+1 and their read-back are enqueued between
        the encode and the decode of pass k, so the host builds pass k+1's
        codes while the device decodes pass k.  Every pass runs every kernel
        over the whole batch; pass k+1's code tables are copied in after pass
        k's decode (stream order).  evs: optional list of per-pass dicts of
        (start, end) events for "hist", "copy" (end only), "enc" and "dec";
        the host build time of each pass is stored under "host"."""
        hc, torch = self.hc, self.torch

        def mark(k, name, i):
            if evs is not None and name in evs[k]:
                evs[k][name][i].record()

        def count(k):
            mark(k, "hist", 0)
            hc.hc_histogram_batch(self.hist_items, self.hist_ws)
            mark(k, "hist", 1)
            self.hist_host.copy_(self.hist, non_blocking=True)
            mark(k, "copy", 1)
            ready = torch.cuda.Event()
            ready.record()
            return ready

        ready = count(0)
        for k in range(steps):
            ready.synchronize()  # pass k's counts are on the host
            t1 = time.perf_counter()
            self.cbset.build(self.hist_host.numpy().view("uint64"))
            if evs is not None and "copy" in evs[k]:
                evs[k]["host"] = time.perf_counter() - t1
            mark(k, "enc", 0)
            hc.hc_encode_batch(self.enc_items, self.B, self.S, self.ws, self.err)
            mark(k, "enc", 1)
            if k + 1 < steps:
                ready = count(k + 1)
            mark(k, "dec", 0)
            hc.hc_decode_batch(self.dec_items, self.B, self.S, self.ws, self.err)
            mark(k, "dec", 1)

    def step_by_kernel(self, ev):
        """The same pass with the encoder's three steps issued as separate calls
        (one kernel each), HIP events around every kernel."""
        hc, torch = self.hc, self.torch
        it, B, S, ws, err = self.enc_items, self.B, self.S, self.ws, self.err
        ev["k_hist"][0].record()
        hc.hc_histogram_batch(self.hist_items, self.hist_ws)
        ev["k_hist"][1].record()
        self.hist_host.copy_(self.hist, non_blocking=True)
        torch.cuda.current_stream().synchronize()
        self.cbset.build(self.hist_host.numpy().view("uint64"))
        for name, fn in (("k_count", hc.hc_encode_lengths_batch), ("k_offsets", hc.hc_encode_offsets_batch),
                         ("k_encode", hc.hc_encode_pack_batch)):
            ev[name][0].record()
            fn(it, B, S, ws, err)
            ev[name][1].record()
        ev["k_decode"][0].record()
        hc.hc_decode_batch(self.dec_items, B, S, ws, err)
        ev["k_decode"][1].record()


KERNELS = ("k_hist", "k_count", "k_offsets", "k_encode", "k_decode")
# the device functions a decode call may launch (one launch per call and kind)
DECODE_KERNELS = ("k_decode_ring", "k_decode_stage", "k_decode")


def kernel_times(w, torch, np, reps=20, warmup=3):
    """Per-kernel GPU time (ms): HIP events recorded around each launch on the
    stream the library launches on (torch's current stream); warm-ups, then
    'reps' passes."""
    E = torch.cuda.Event
    out = {k: [] for k in KERNELS}
    for r in range(warmup + reps):
        ev = {k: (E(enable_timing=True), E(enable_timing=True)) for k in KERNELS}
        w.step_by_kernel(ev)
        torch.cuda.synchronize()
        if r >= warmup:
            for k in KERNELS:
                out[k].append(ev[k][0].elapsed_time(ev[k][1]))
    return out


TUNE_CANDIDATES = ([{"block_size": B, "sub_block": 128, "encode_tile_loads": q} for B in (4096, 16384, 65536, 262144)
                    for q in (0, 2)] +
                   [{"block_size": B, "sub_block": 1024, "encode_tile_loads": 0} for B in (16384, 65536, 262144)])


def autotune_step(hc, synth, torch, nseg: int, steps: int = 3):
    """The autotuner (paper_1107_1525_amd.autotune) over block size, index
    stride and encode tile on nseg segments of the mixed workload: each
    candidate's whole step (counts, codes, encode, decode) timed over
    'steps' passes after one warm-up, its round trip checked.  Cached per
    device and workload; the winner is what the timed run uses."""
    from paper_1107_1525_amd.autotune import Autotuner, device_key

    def measure(c):
        hc.hc_set_tuning(c["encode_tile_loads"])
        try:
            w = Workload(hc, synth, torch, nseg, c["block_size"], c["sub_block"])
            w.run(1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            w.run(steps)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / steps
            if hc.read_error(w.err):
                raise hc.HcError(hc.read_error(w.err), "autotune")
            if not torch.equal(w.y, w.x):
                raise RuntimeError("round trip failed")
            del w
            return t
        finally:
            torch.cuda.empty_cache()
            hc.hc_set_tuning(0)

    tuner = Autotuner()
    dev = device_key(torch)
    key = f"{WORKLOAD}/sample{nseg}"
    best, table, cached = tuner.tune(dev, key, TUNE_CANDIDATES, measure)
    n = nseg * synth.WORKLOADS[WORKLOAD]["segment"]
    return {"best": best, "device": dev, "workload": key, "cached": cached,
            "table": [{**r["candidate"], **({"GBps": round(n / r["seconds"] / 1e9, 1)} if "seconds" in r
                                            else {"error": r.get("error")})} for r in table]}


def subset_times(w, segs, torch, np, reps=10, warmup=2):
    """The encoder's three steps and the decode of the segments 'segs' alone,
    through the batched calls on that subset (same buffers), HIP events
    around every call: mean ms per call."""
    hc = w.hc
    E = torch.cuda.Event
    e_it, d_it = hc.make_items(len(segs)), hc.make_items(len(segs))
    for j, t in enumerate(segs):
        hc.set_item(e_it, j, x=w.xs(t), dcb=w.dcb[t], out=w.outs(t), block_off=w.off[t], sub_idx=w.subs(t))
        hc.set_item(d_it, j, x=w.outs(t), n=w.seg, in_bytes=w.C[t], dcb=w.dcb[t], out=w.ys(t),
                    block_off=w.off[t], sub_idx=w.subs(t))
    steps = (("k_count", lambda: hc.hc_encode_lengths_batch(e_it, w.B, w.S, w.ws, w.err)),
             ("k_offsets", lambda: hc.hc_encode_offsets_batch(e_it, w.B, w.S, w.ws, w.err)),
             ("k_encode", lambda: hc.hc_encode_pack_batch(e_it, w.B, w.S, w.ws, w.err)),
             ("k_decode", lambda: hc.hc_decode_batch(d_it, w.B, w.S, w.ws, w.err)))
    t = {k: [] for k, _ in steps}
    for r in range(warmup + reps):
        ev = {k: (E(enable_timing=True), E(enable_timing=True)) for k, _ in steps}
        for k, fn in steps:
            ev[k][0].record()
            fn()
            ev[k][1].record()
        torch.cuda.synchronize()
        if r >= warmup:
            for k, _ in steps:
                t[k].append(ev[k][0].elapsed_time(ev[k][1]))
    return {k: float(np.mean(v)) for k, v in t.items()}


def subset_bytes(w, segs, np):
    """Algorithmic bytes of each step over the segments 'segs'."""
    n = w.seg * len(segs)
    C = sum(w.C[j] for j in segs)
    side = (8 * (w.nb + 1) + 4 * w.nsub) * len(segs)
    complete8 = all(bool(np.all(np.asarray(w.dcb[j].host.lengths) == 8)) for j in segs)
    return n, C, complete8, {"k_count": 0 if complete8 else n, "k_offsets": 8 * (w.nb + 1) * len(segs),
                             "k_encode": n + C + side, "k_decode": C + n + side}


def class_launch_times(w, torch, np):
    """The mixed workload's two launch classes apart, each one call over its
    own segments: the complete 8-bit codes (uniform segments: the encoder's
    and the decoder's copy forms) and the rest (skewed and fp32 segments,
    whose codes fall in one class: one length pass, one packing launch, one
    table-decoder launch, the very launches of the whole step).  Each call is
    then a single kernel launch, so these are per-launch times that a
    kernel trace of the whole step reproduces."""
    c8 = [t for t in range(w.nseg) if bool(np.all(np.asarray(w.dcb[t].host.lengths) == 8))]
    rest = [t for t in range(w.nseg) if t not in set(c8)]
    out = {}
    for name, segs in (("copy", c8), ("table", rest)):
        if not segs:
            continue
        ms = subset_times(w, segs, torch, np)
        n, C, _, alg = subset_bytes(w, segs, np)
        out[name] = {"segments": len(segs), "bytes": n, "compressed": C, "ms": ms, "alg": alg}
    return out


def kind_kernel_times(w, synth, torch, np, reps=10, warmup=2):
    """The same workload's segments of one kind at a time, through the
    batched calls on that subset (same buffers): the encoder's three launches
    and the decode launch of each kind, HIP events around every launch.  The
    decode of the uniform segments (complete 8-bit codes) is the decoder's
    copy launch, that of the others its table-decode launch, so this also
    times the two launches of the whole workload's decode call apart."""
    out = {}
    for kind in synth.SEGMENT_KINDS:
        segs = [t for t in range(w.nseg) if synth.mixed_kind(t) == kind]
        if not segs:
            continue
        ms = subset_times(w, segs, torch, np, reps=reps, warmup=warmup)
        n, C, complete8, alg = subset_bytes(w, segs, np)
        out[kind] = {
            "segments": len(segs), "bytes": n, "ratio": round(C / n, 5),
            "max_len": max(int(w.dcb[j].max_len) for j in segs),
            "decode_kernel": "k_decode_ring (copy form)" if complete8 else "k_decode_stage",
            **{k: {"avg_ms": round(v, 4), "ms_per_GiB": round(v * (1 << 30) / n, 4),
                   "GBps_alg": round(alg[k] / (v * 1e-3) / 1e9, 1) if alg[k] else None,
                   "pct_hbm": round(100 * alg[k] / (v * 1e-3) / 1e9 / HBM_PEAK_GBPS, 1) if alg[k] else None}
               for k, v in ms.items()},
        }
    return out


def single_stream_bench(hc, synth, torch, np, name: str, S: int, reps: int = 20, warmup: int = 3):
    """One buffer, one codebook: compress (counts, their read-back, the host
    code build and table refresh, the three encode launches) and decompress
    (the decode), timed per call; plus the header walk that rebuilds the
    offset table of a stream kept without it.  Median and p10/p90 of 'reps'
    calls after 'warmup'; the round trip is checked."""
    spec = synth.WORKLOADS[name]
    n, B = spec["n"], spec["block"]
    seed = synth.derive_seed(spec["config_id"], 0)
    x = synth.zipf_bytes_torch(n, spec["s"], seed) if n >= (64 << 20) else \
        torch.from_numpy(synth.zipf_bytes(n, spec["s"], seed)).cuda()
    nb = hc.num_blocks(n, B)
    hist = torch.zeros(256, dtype=torch.int64, device="cuda")
    hist_host = torch.zeros(256, dtype=torch.int64).pin_memory()
    hc.hc_histogram(x, out=hist)
    cb = hc.hc_build_codebook(hist.cpu().numpy().view(np.uint64))
    dcb = hc.DeviceCodebook(cb)
    cap = (hc.hc_encode_bound(n, B, cb.max_len) + 255) // 256 * 256
    out = torch.empty(cap, dtype=torch.uint8, device="cuda")
    off = torch.empty(nb + 1, dtype=torch.int64, device="cuda")
    off2 = torch.empty(nb + 1, dtype=torch.int64, device="cuda")
    sub = torch.empty(max(hc.hc_sub_index_entries(n, B, S), 1), dtype=torch.int32, device="cuda")
    ws = torch.empty(max(hc.hc_encode_workspace_bytes(n, B), 16), dtype=torch.uint8, device="cuda")
    y = torch.empty(n, dtype=torch.uint8, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    E = torch.cuda.Event
    tc, td, tw = [], [], []
    for r in range(warmup + reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hc.hc_histogram(x, out=hist)
        hist_host.copy_(hist, non_blocking=True)
        torch.cuda.current_stream().synchronize()
        c = hc.hc_build_codebook(hist_host.numpy().view(np.uint64))
        dcb.update(c)
        hc.hc_encode_blocks(x, B, dcb, out, off, sub, S, ws, err)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        a, b = E(enable_timing=True), E(enable_timing=True)
        a.record()
        hc.hc_decode_blocks(out, int(off[nb].item()), n, B, dcb, off, sub, S, y, err)
        b.record()
        c1, c2 = E(enable_timing=True), E(enable_timing=True)
        C = int(off[nb].item())
        c1.record()
        hc.hc_walk_blocks(out, C, nb, off2, err)
        c2.record()
        torch.cuda.synchronize()
        if r >= warmup:
            tc.append(1e3 * (t1 - t0))
            td.append(a.elapsed_time(b))
            tw.append(c1.elapsed_time(c2))
    if hc.read_error(err):
        raise hc.HcError(hc.read_error(err), name)
    assert torch.equal(y, x), f"round trip failed ({name})"
    assert torch.equal(off2, off), f"walk differs from the encoder's offsets ({name})"
    side = 8 * (nb + 1) + 4 * hc.hc_sub_index_entries(n, B, S)
    pct = lambda nbytes, ms: round(100 * nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 1)
    q = lambda v: {"p10": round(float(np.percentile(v, 10)), 4), "p50": round(float(np.median(v)), 4),
                   "p90": round(float(np.percentile(v, 90)), 4)}
    mc, md = float(np.median(tc)), float(np.median(td))
    return {
        "workload": name, "bytes": n, "block_size": B, "sub_block": S, "ratio": round(C / n, 5),
        "compress_ms": q(tc), "decompress_ms": q(td),
        "compress_GBps": round(n / (mc * 1e-3) / 1e9, 1), "decompress_GBps": round(n / (md * 1e-3) / 1e9, 1),
        "compress_pct_hbm": pct(3 * n + C + side, mc), "decompress_pct_hbm": pct(C + n + side, md),
        "compress_note": "wall clock: counts + read-back + host code build + table refresh + encode",
        "walk_ms": q(tw), "walk_blocks": nb,
    }


def cpu_baseline(w, oracle, np):
    """The oracle on segments 0..5 (two of each kind, 384 MiB) of the same
    workload: counts, code, block encode and strict decode.  Timed twice: on
    one thread, and block-parallel on every host core the process may use (a
    thread pool over independent blocks; the oracle's C calls release the
    interpreter lock), which is the shape of the paper's multi-core coder."""
    from concurrent.futures import ThreadPoolExecutor

    xs = [w.xs(t).cpu().numpy() for t in range(6)]
    nbytes = sum(x.size for x in xs)
    B = w.B

    def one_thread():
        for x in xs:
            h = oracle.histogram(x)
            L, C = oracle.codebook(h)
            s, off, bits = oracle.encode(x, B, L, C)
            y = oracle.decode(s, x.size, B, L)
            assert np.array_equal(y, x)

    # every core in the affinity mask, up to the 16 CPUs a one-GPU job is given on the GPU machine
    available = len(os.sched_getaffinity(0))
    cores = min(16, available)

    def block_parallel(pool):
        for x in xs:
            blocks = [x[i:i + B] for i in range(0, x.size, B)]
            h = sum(pool.map(oracle.histogram, blocks))
            L, C = oracle.codebook(h)
            enc = list(pool.map(lambda b: oracle.encode(b, B, L, C)[0], blocks))
            dec = list(pool.map(lambda sb: oracle.decode(sb[0], sb[1].size, B, L), zip(enc, blocks)))
            assert all(np.array_equal(d, b) for d, b in zip(dec, blocks))

    t0 = time.perf_counter()
    one_thread()
    t1 = time.perf_counter() - t0
    with ThreadPoolExecutor(cores) as pool:
        t0 = time.perf_counter()
        block_parallel(pool)
        tp = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {
        "value": round(nbytes / tp / 1e9, 4),
        "unit": "GB/s",
        "cores": cores,
        "cores_available": available,
        "cpu": model,
        "kind": "oracle",
        "sample": f"segments 0-5 (uniform, skewed, fp32, twice) of the 4 GiB mixed workload, {nbytes >> 20} MiB, "
                  f"B={B}: counts + code + block encode + strict decode, block-parallel over {cores} threads",
        "seconds": round(tp, 2),
        "single_core_GBps": round(nbytes / t1 / 1e9, 4),
        "single_core_seconds": round(t1, 2),
    }


def load_traffic(kernel: str, B: int, S: int):
    """HBM bytes per launch from committed rocprofv3 PMC summaries, if they
    were taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{WORKLOAD}_B{B}_S{S}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def _loguniform_sizes(rng, count, lo, hi):
    import numpy as np

    return [int(v) for v in np.exp(rng.uniform(np.log(lo), np.log(hi), size=count))]


def batched_bench(hc, synth, torch, np, count: int, B: int, S: int, reps: int = 5):
    """Independent buffers with their own codebooks (sizes log-uniform in
    1 KiB-64 MiB, Zipf s ~ U[0.8, 1.6]): one batched launch per phase, the
    same batched calls replayed from a HIP graph, and one buffer per launch,
    on the same buffers with the same results.  Inputs, streams and decoded
    outputs live in three arenas; if the device cannot hold them all, the
    batch keeps as many of the buffers (in order) as fit, and says so."""
    asked = count
    rng = np.random.default_rng(synth.derive_seed(4, 0))
    sizes = _loguniform_sizes(rng, count, 1 << 10, 64 << 20)
    s_of = [float(rng.uniform(0.8, 1.6)) for _ in range(count)]
    r256 = lambda v: (v + 255) // 256 * 256
    # inputs + streams at the loosest bound (codes of <= 16 bits: 2 bytes per
    # symbol) + decoded outputs, with room to spare for the workspace
    free = torch.cuda.mem_get_info()[0]
    kept, need = 0, 0
    for n in sizes:
        step = r256(n) * 2 + r256(2 * n + 8 * hc.num_blocks(n, B) + 64)
        if need + step > 0.85 * free:
            break
        need += step
        kept += 1
    sizes, s_of = sizes[:kept], s_of[:kept]
    count = kept
    base = [0]
    for n in sizes:
        base.append(base[-1] + r256(n))
    total = sum(sizes)
    x_arena = torch.empty(base[-1], dtype=torch.uint8, device="cuda")
    xs = [x_arena[base[k]:base[k] + n] for k, n in enumerate(sizes)]
    for k, n in enumerate(sizes):
        synth.zipf_bytes_torch(n, s_of[k], synth.derive_seed(4, k + 1), out=xs[k])
    hist = torch.empty((count, 256), dtype=torch.int64, device="cuda")
    items = hc.make_items(count)
    for k, x in enumerate(xs):
        hc.set_item(items, k, x=x, hist=hist[k])
    hws = torch.empty(max(hc.hc_batch_workspace_bytes(items, B), 256), dtype=torch.uint8, device="cuda")
    hc.hc_histogram_batch(items, hws)
    cbset = hc.CodebookSet(count)
    dcbs = cbset.build(hist.cpu().numpy().view(np.uint64))
    caps = [r256(hc.hc_encode_bound(n, B, d.max_len)) for n, d in zip(sizes, dcbs)]
    obase = [0]
    for c in caps:
        obase.append(obase[-1] + c)
    o_arena = torch.empty(obase[-1], dtype=torch.uint8, device="cuda")
    outs = [o_arena[obase[k]:obase[k] + caps[k]] for k in range(count)]
    y_arena = torch.zeros(base[-1], dtype=torch.uint8, device="cuda")
    ys = [y_arena[base[k]:base[k] + n] for k, n in enumerate(sizes)]
    nbs = [hc.num_blocks(n, B) for n in sizes]
    off_arena = torch.empty(sum(nb + 1 for nb in nbs), dtype=torch.int64, device="cuda")
    ob = np.concatenate([[0], np.cumsum([nb + 1 for nb in nbs])])
    offs = [off_arena[ob[k]:ob[k + 1]] for k in range(count)]
    nsub = [max(hc.hc_sub_index_entries(n, B, S), 1) if S else 0 for n in sizes]
    sb = np.concatenate([[0], np.cumsum(nsub)])
    sub_arena = torch.empty(max(int(sb[-1]), 1), dtype=torch.int32, device="cuda")
    subs = [sub_arena[sb[k]:sb[k + 1]] if S else None for k in range(count)]
    enc_items = hc.make_items(count)
    for k in range(count):
        hc.set_item(enc_items, k, x=xs[k], dcb=dcbs[k], out=outs[k], block_off=offs[k], sub_idx=subs[k])
    ws = torch.empty(hc.hc_batch_workspace_bytes(enc_items, B), dtype=torch.uint8, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    hc.hc_encode_batch(enc_items, B, S, ws, err)
    C = [int(v) for v in off_arena[torch.from_numpy(ob[1:] - 1).cuda()].cpu()]
    dec_items = hc.make_items(count)
    for k in range(count):
        hc.set_item(dec_items, k, x=outs[k], n=sizes[k], in_bytes=C[k], dcb=dcbs[k], out=ys[k], block_off=offs[k],
                    sub_idx=subs[k])
    single_ws = torch.empty(max(hc.hc_encode_workspace_bytes(max(sizes), B), 16), dtype=torch.uint8, device="cuda")

    def batched():
        hc.hc_histogram_batch(items, hws)
        hc.hc_encode_batch(enc_items, B, S, ws, err)
        hc.hc_decode_batch(dec_items, B, S, ws, err)

    def plain():
        for k in range(count):
            hc.hc_histogram(xs[k], out=hist[k])
            hc.hc_encode_blocks(xs[k], B, dcbs[k], outs[k], offs[k], subs[k], S, single_ws, err)
            hc.hc_decode_blocks(outs[k], C[k], sizes[k], B, dcbs[k], offs[k], subs[k], S, ys[k], err)

    def timed(fn, n_reps):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(n_reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return ts

    res = {"batched": timed(batched, reps)}
    assert hc.read_error(err) == 0 and torch.equal(y_arena, x_arena), "batched round trip"
    y_arena.zero_()
    res["plain"] = timed(plain, max(2, reps // 2))
    assert hc.read_error(err) == 0 and torch.equal(y_arena, x_arena), "plain round trip"
    # the batched calls captured once in a HIP graph, then replayed
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=side):
        batched()
    y_arena.zero_()
    torch.cuda.synchronize()
    res["graph"] = timed(g.replay, reps)
    assert hc.read_error(err) == 0 and torch.equal(y_arena, x_arena), "graph replay round trip"
    out = {"buffers": count, "buffers_asked": asked, "bytes": total, "compressed_bytes": int(sum(C)), "sizes": "log-uniform 1 KiB-64 MiB",
           "data": "Zipf s~U[0.8,1.6], one codebook per buffer", "block_size": B, "sub_block": S,
           "phases": "counts + encode + decode per pass (codebooks resident); graph: the same three batched calls"}
    for name, ts in res.items():
        med = float(np.median(ts))
        out[f"{name}_GBps"] = round(total / med / 1e9, 2)
        out[f"{name}_ms"] = {"p10": round(1e3 * float(np.percentile(ts, 10)), 3), "p50": round(1e3 * med, 3),
                             "p90": round(1e3 * float(np.percentile(ts, 90)), 3)}
    return out


def serve_bench(hc, synth, torch, np, count: int, B: int, S: int, warmup: int = 500, check_every: int = 8):
    """The serving loop (paper_1107_1525_amd.serve) against the plain form
    (one request per launch, one at a time, first come first served): 50/50
    compress/decompress, sizes log-uniform 4 KiB-256 MiB, each request's
    bytes of one of the mixed workload's three kinds.  Saturation (every
    request waiting at the start: aggregate GB/s of each form), then the
    same Poisson arrivals at 0.5 and 0.8 of the plain form's capacity fed to
    both: p50/p99 of completion minus arrival (queueing included), over the
    requests after the first 'warmup'.  Arrival times start once the server
    is built and every request queued; garbage collection is off inside
    every timed loop of both forms.  A request's input is a slice of a
    512 MiB pool of its kind (so the inputs need no more memory than the
    pools); decompress requests are encoded beforehand, each its own
    stream; results are dropped as they retire except every
    'check_every'-th, which is checked (a round trip, and the same bytes as
    the plain form)."""
    from paper_1107_1525_amd.serve import Request, Server, percentile

    rng = np.random.default_rng(synth.derive_seed(5, 0))
    sizes = _loguniform_sizes(rng, count, 4 << 10, 256 << 20)
    is_comp = rng.random(count) < 0.5
    kinds = rng.integers(0, 3, size=count)
    pool_n = 512 << 20
    pools = [synth.segment_bytes_torch(k, pool_n, synth.derive_seed(5, 1 + i)) for i, k in enumerate(synth.SEGMENT_KINDS)]
    offs = [int(rng.integers(0, (pool_n - n) // 256 + 1)) * 256 for n in sizes]
    data = [pools[kinds[k]][offs[k]:offs[k] + sizes[k]] for k in range(count)]
    encs = [None if is_comp[k] else hc.compress(data[k], B, sub_block=S) for k in range(count)]
    torch.cuda.synchronize()
    total = sum(sizes)
    say = lambda m: print(f"[bench] serving: {m}", file=sys.stderr, flush=True)
    say(f"{count} requests, {total / 1e9:.1f} GB, decompress inputs encoded")

    def plain_one(k):
        if is_comp[k]:
            e = hc.compress(data[k], B, sub_block=S)
        else:
            e = hc.decompress(encs[k])
        torch.cuda.synchronize()
        return e

    checks = {}

    def make_server():
        def done(r):
            lat[r.rid] = r.latency
            if r.rid % check_every == 0:
                checks[r.rid] = r.result
            elif r.kind == "compress":
                srv.recycle(r.result)
            r.result = None
        lat = {}
        srv = Server(block_size=B, sub_block=S, hbm_budget=32 << 30, tables=4096, on_done=done)
        return srv, lat

    class quiet:
        """No garbage collection inside a timed loop (a full collection of
        this process's objects pauses it for tens of ms): collected before,
        re-enabled after, for both forms alike."""

        def __enter__(self):
            gc.collect()
            gc.disable()

        def __exit__(self, *exc):
            gc.enable()

    def served(gaps):
        """Serves every request, the k-th arriving sum(gaps[:k+1]) seconds
        after the server is built and every request queued (setup is not
        counted as waiting)."""
        srv, lat = make_server()
        reqs = []
        for k in range(count):
            req = (Request("compress", data=data[k], arrival=float("inf")) if is_comp[k] else
                   Request("decompress", encoded=encs[k], arrival=float("inf")))
            reqs.append(srv.submit(req))  # rid == k
        with quiet():
            start = time.perf_counter() + 0.01
            for r, a in zip(reqs, start + np.cumsum(gaps)):
                r.arrival = float(a)
            srv.run_until_idle()
        assert len(lat) == count
        return srv, [lat[k] for k in range(count)], start

    def verify():
        for k, res in checks.items():
            if is_comp[k]:
                ref = hc.compress(data[k], B, sub_block=S)
                assert torch.equal(res.stream, ref.stream) and torch.equal(res.block_off, ref.block_off), k
                assert torch.equal(hc.decompress(res), data[k]), k
            else:
                assert torch.equal(res, data[k]), k
        n = len(checks)
        checks.clear()
        return n

    # saturation
    for k in range(min(count, 16)):
        plain_one(k)  # warm-up
    with quiet():
        t0 = time.perf_counter()
        for k in range(count):
            plain_one(k)
        plain_s = time.perf_counter() - t0
    plain_rate = total / plain_s
    say(f"plain at saturation {plain_rate / 1e9:.1f} GB/s")
    srv, _, t0 = served(np.zeros(count))
    served_s = time.perf_counter() - t0
    checked = verify()
    say(f"served at saturation {total / served_s / 1e9:.1f} GB/s ({checked} results checked)")
    out = {
        "requests": count, "warmup_requests": warmup, "bytes": total, "sizes": "log-uniform 4 KiB-256 MiB",
        "mix": "50/50 compress/decompress", "data": "each request one of uniform/skewed/fp32 bytes",
        "block_size": B, "sub_block": S, "hbm_budget": 32 << 30,
        "saturation_GBps": {"served": round(total / served_s / 1e9, 2), "plain": round(plain_rate / 1e9, 2)},
        "loads": [],
    }
    ms = lambda v: round(v * 1e3, 3)
    for rho in (0.5, 0.8):
        gaps = rng.exponential(np.mean(sizes) / (rho * plain_rate), size=count)
        lat_plain = []
        with quiet():
            start = time.perf_counter() + 0.01
            arr = start + np.cumsum(gaps)
            for k in range(count):
                while time.perf_counter() < arr[k]:
                    pass
                plain_one(k)
                lat_plain.append(time.perf_counter() - arr[k])
        say(f"plain at {rho} of capacity done")
        srv, lat, _ = served(gaps)
        checked += verify()
        lp, ls = lat_plain[warmup:], lat[warmup:]
        say(f"served at {rho} of capacity: p99 {percentile(ls, 99) * 1e3:.2f} ms (plain {percentile(lp, 99) * 1e3:.2f} ms)")
        out["loads"].append({
            "offered": f"{rho} x plain capacity ({rho * plain_rate / 1e9:.2f} GB/s), Poisson",
            "served_p50_ms": ms(percentile(ls, 50)), "served_p99_ms": ms(percentile(ls, 99)),
            "plain_p50_ms": ms(percentile(lp, 50)), "plain_p99_ms": ms(percentile(lp, 99)),
            "iterations": srv.iterations, "max_inflight_requests": srv.max_inflight_requests,
            "table_growths": srv.table_growths,
        })
    out["checked_results"] = checked
    return out


def kernel_name(full: str) -> str:
    """A rocprofv3 kernel name without its parameter list, return type and
    anonymous-namespace prefix (the probes live in one)."""
    return full.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")


def _pmc_per_kernel(root: str, counter: str):
    """Mean counter value (KiB) per dispatch, by kernel, from rocprofv3 CSVs."""
    import csv
    import glob

    vals = {}
    for f in glob.glob(os.path.join(root, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] != counter:
                continue
            name = kernel_name(r["Kernel_Name"])
            vals.setdefault(name, []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in vals.items()}


def traffic_summary(root: str, B: int, S: int, out_dir: str = None):
    """Per-launch HBM traffic of each codec kernel.  Each counter is scaled by
    what it reads for a plain 1 GiB device copy (bytes known exactly)."""
    copy_bytes = 1 << 30
    fetch, write = _pmc_per_kernel(os.path.join(root, "fetch"), "FETCH_SIZE"), \
        _pmc_per_kernel(os.path.join(root, "write"), "WRITE_SIZE")
    cf = _pmc_per_kernel(os.path.join(root, "copy_fetch"), "FETCH_SIZE")
    cw = _pmc_per_kernel(os.path.join(root, "copy_write"), "WRITE_SIZE")
    # the probe's 1 GiB copy (its read probe fetches as much but writes nothing)
    copy_name = next((k for k in cf if "k_probe_copy" in k), None) or max(cf, key=cf.get)
    f_scale = copy_bytes / (cf[copy_name] * 1024.0)
    w_scale = copy_bytes / (cw[copy_name] * 1024.0)
    # cross-check of the fetch scale on the read probe (1 GiB read, nothing
    # written, another access pattern): the same factor should come out
    read_name = next((k for k in cf if "k_probe_read" in k), None)
    f_scale_read = copy_bytes / (cf[read_name] * 1024.0) if read_name else None
    # a decode call runs two instances of k_decode_ring (the copy form for
    # complete 8-bit codes, the ring decoder for the rest), each once per
    # call: the instances of a kernel are summed, per call
    out = {}
    for k in fetch:
        short = k.split("::")[-1].split("<")[0]
        if not short.startswith("k_") or short.startswith("k_probe"):  # codec kernels only
            continue
        rec = {
            "kernel": k, "fetch_kib_per_dispatch": round(fetch[k], 1), "write_kib_per_dispatch": round(write.get(k, 0.0), 1),
            "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4),
            "fetch_scale_read_probe": None if f_scale_read is None else round(f_scale_read, 4),
            "bytes_per_launch": int(fetch[k] * 1024 * f_scale + write.get(k, 0.0) * 1024 * w_scale),
            "kernel_source_hash": kernel_source_hash(), "workload": WORKLOAD, "block_size": B, "sub_block": S,
            "copy_kernel": copy_name, "copy_bytes": copy_bytes,
            "commands": [
                f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT/fetch -o run -- "
                f"python -u bench.py --only-step --steps 1 --warmup 1 --block {B} --sub-block {S} --tile-loads 0",
                f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT/write -o run -- "
                f"python -u bench.py --only-step --steps 1 --warmup 1 --block {B} --sub-block {S} --tile-loads 0",
                "rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT/copy_fetch -o run -- "
                "python -u bench.py --copy-probe",
                "rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT/copy_write -o run -- "
                "python -u bench.py --copy-probe",
                f"python bench.py --traffic-summary OUT --block {B} --sub-block {S}",
            ],
            "OUT": "the directory the four rocprofv3 runs wrote (any path)",
        }
        path = os.path.join(out_dir or os.path.join(ROOT, "profiles"), f"traffic_{short}_{WORKLOAD}_B{B}_S{S}.json")
        if short in out:  # another instance of the same kernel in each call: add it
            prev = out[short]
            rec["kernel"] = prev["kernel"] + " + " + rec["kernel"]
            rec["fetch_kib_per_dispatch"] = round(prev["fetch_kib_per_dispatch"] + rec["fetch_kib_per_dispatch"], 1)
            rec["write_kib_per_dispatch"] = round(prev["write_kib_per_dispatch"] + rec["write_kib_per_dispatch"], 1)
            rec["bytes_per_launch"] += prev["bytes_per_launch"]
        out[short] = rec
        with open(path, "w") as f:
            json.dump(rec, f, indent=1)
    print(json.dumps(out, indent=1))
    return out


def trace_summary(root: str, B: int, S: int):
    """Markdown table of the codec kernels in a rocprofv3 kernel trace of
    `bench.py --only-step`: calls and duration per kernel instance over all
    dispatches, and over the dispatches no other codec kernel overlapped
    (the launches the bench times one at a time; in the step itself a call's
    class launches run side by side and stretch each other)."""
    import csv
    import glob

    def codec(name):
        return kernel_name(name).split("::")[-1].startswith(("k_", "hc::k_")) or "hc::k_" in name

    rows = []
    for f in glob.glob(os.path.join(root, "**", "*kernel_trace.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if codec(r["Kernel_Name"]):
                rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), kernel_name(r["Kernel_Name"])))
    rows.sort()
    alone, running = [], -1  # running: the latest end among earlier-starting dispatches
    for i, (a, b, nm) in enumerate(rows):
        nxt = rows[i + 1][0] if i + 1 < len(rows) else 1 << 62  # sorted by start: the next start is the earliest
        alone.append(running <= a and nxt >= b)
        running = max(running, b)
    by = {}
    for (a, b, nm), al in zip(rows, alone):
        d = by.setdefault(nm, {"all": [], "alone": []})
        d["all"].append((b - a) / 1e3)
        if al:
            d["alone"].append((b - a) / 1e3)
    lines = [f"| kernel | calls | avg us | min us | max us | alone calls | alone avg us |", "|---|---|---|---|---|---|---|"]
    for nm, d in sorted(by.items(), key=lambda kv: -sum(kv[1]["all"])):
        al = d["alone"]
        lines.append(f"| `{nm.replace('hc::', '')}` | {len(d['all'])} | {sum(d['all']) / len(d['all']):.2f} | "
                     f"{min(d['all']):.2f} | {max(d['all']):.2f} | {len(al)} | "
                     f"{(sum(al) / len(al)) if al else float('nan'):.2f} |")
    print("\n".join(lines))


def sq_table(root: str, synth, args):
    """Per-kind SQ counter table from rocprofv3 --pmc runs of --per-kind.

    Each kind runs the workload set-up, then warm-up + timed passes, each
    ending with one decode launch; the last launch of each kernel before a
    kind's final decode is that kind's timed launch.  VALU and LDS are wave
    instructions x 64 lanes per input symbol; conflict is
    SQ_LDS_BANK_CONFLICT / SQ_ACTIVE_INST_LDS; wait, wait-issue and active are
    SQ_WAIT_ANY, SQ_WAIT_INST_ANY and SQ_ACTIVE_INST_ANY over SQ_WAVE_CYCLES."""
    import csv
    import glob

    per_kind = args.warmup + args.steps
    symbols = args.segments * synth.WORKLOADS[WORKLOAD]["segment"]
    vals = {}  # (kind index, kernel) -> counter -> value
    for f in sorted(glob.glob(os.path.join(root, "**", "*counter_collection.csv"), recursive=True)):
        disp = {}
        for r in csv.DictReader(open(f)):
            d = disp.setdefault(int(r["Dispatch_Id"]), {"name": kernel_name(r["Kernel_Name"])})
            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        kind, decodes, last = 0, 0, {}
        for i in sorted(disp):
            name = disp[i]["name"]
            short = name.split("::")[-1].split("<")[0]
            if short in ("k_count", "k_encode") + DECODE_KERNELS:
                last[name] = disp[i]
            if short in DECODE_KERNELS:
                decodes += 1
                if decodes == per_kind:
                    for k, c in last.items():
                        vals.setdefault((kind, k), {}).update({n: v for n, v in c.items() if n != "name"})
                    kind, decodes, last = kind + 1, 0, {}
    rows = ["| kind | kernel | VALU / symbol | LDS / symbol | conflict / LDS active | wait | wait issue | active |",
            "|---|---|---|---|---|---|---|---|"]
    order = {"k_count": 0, "k_encode": 1, **{k: 2 for k in DECODE_KERNELS}}
    for (kind, k) in sorted(vals, key=lambda t: (t[0], order[t[1].split("::")[-1].split("<")[0]])):
        c = vals[(kind, k)]
        g = lambda n: c.get(n, float("nan"))
        cyc = g("SQ_WAVE_CYCLES")
        rows.append(f"| {synth.SEGMENT_KINDS[kind]} | `{k.split('::')[-1]}` | {64 * g('SQ_INSTS_VALU') / symbols:.2f} | "
                    f"{64 * g('SQ_INSTS_LDS') / symbols:.2f} | {g('SQ_LDS_BANK_CONFLICT') / g('SQ_ACTIVE_INST_LDS'):.2f} | "
                    f"{g('SQ_WAIT_ANY') / cyc:.2f} | {g('SQ_WAIT_INST_ANY') / cyc:.2f} | {g('SQ_ACTIVE_INST_ANY') / cyc:.2f} |")
    print("\n".join(rows))


def per_kind_bench(hc, synth, torch, np, args):
    """The step on args.segments segments of one kind at a time: each
    kernel's average time over args.steps passes (HIP events around every
    launch) and its rate in algorithmic bytes, one JSON line per kind."""
    for kind in synth.SEGMENT_KINDS:
        print(f"[bench] {kind}: {args.segments} x 64 MiB", file=sys.stderr, flush=True)
        w = Workload(hc, synth, torch, args.segments, args.block, args.sub_block, kind=kind)
        kt = kernel_times(w, torch, np, reps=args.steps, warmup=args.warmup)
        if hc.read_error(w.err):
            raise hc.HcError(hc.read_error(w.err), kind)
        assert torch.equal(w.y, w.x), f"round trip failed ({kind})"
        n, C = w.n, sum(w.C)
        side = 8 * (w.nb + 1) * w.nseg + 4 * w.nsub * w.nseg
        complete8 = all(bool(np.all(np.asarray(d.host.lengths) == 8)) for d in w.dcb)
        alg = {"k_hist": n + 8 * 256 * w.nseg, "k_count": 0 if complete8 else n, "k_offsets": 8 * (w.nb + 1) * w.nseg,
               "k_encode": n + C + side, "k_decode": C + n + side}
        kernels = {}
        for k in KERNELS:
            ms = float(np.mean(kt[k]))
            kernels[k] = {"avg_ms": round(ms, 4), "GBps_alg": round(alg[k] / (ms * 1e-3) / 1e9, 1)}
        print(json.dumps({"kind": kind, "bytes": n, "ratio": round(C / n, 5),
                          "max_len": [min(d.max_len for d in w.dcb), max(d.max_len for d in w.dcb)],
                          "block_size": args.block, "sub_block": args.sub_block, "kernels": kernels}), flush=True)
        del w
        torch.cuda.empty_cache()


def host_pipeline_bench(hc, synth, torch, np, nseg: int, B: int, S: int, reps: int = 3):
    """The mixed workload held in pinned host memory, through the chunked
    host pipeline (paper_1107_1525_amd.hostpipe): wall-clock compress and
    decompress rates including every host<->device copy, the round trip
    checked, and plain pinned copies of 1 GiB each way (the PCIe bound)."""
    from paper_1107_1525_amd.hostpipe import HostPipeline

    seg = synth.WORKLOADS[WORKLOAD]["segment"]
    n = seg * nseg
    xh = torch.empty(n, dtype=torch.uint8).pin_memory()
    for t in range(nseg):
        xh[t * seg:(t + 1) * seg].copy_(synth.segment_bytes_torch(synth.mixed_kind(t), seg, synth.derive_seed(3, t)))
    pipe = HostPipeline(B, S, chunk_bytes=seg, slots=3)
    enc = pipe.compress(xh)  # warm-up, and the output buffers
    y = pipe.decompress(enc)
    assert torch.equal(y, xh), "host pipeline round trip failed"
    tc, td = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        enc = pipe.compress(xh, out=enc.data)
        tc.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        pipe.decompress(enc, y)
        td.append(time.perf_counter() - t0)
    assert torch.equal(y, xh), "host pipeline round trip failed (timed)"
    # plain pinned copies, 1 GiB each way, on a side stream
    g = 1 << 30
    hbuf = torch.empty(g, dtype=torch.uint8).pin_memory()
    dbuf = torch.empty(g, dtype=torch.uint8, device="cuda")
    st = torch.cuda.Stream()
    rates = {}
    for name, fn in (("h2d", lambda: dbuf.copy_(hbuf, non_blocking=True)),
                     ("d2h", lambda: hbuf.copy_(dbuf, non_blocking=True))):
        with torch.cuda.stream(st):
            fn()
            st.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            st.synchronize()
        rates[name] = reps * g / (time.perf_counter() - t0) / 1e9
    del hbuf, dbuf
    return {
        "bytes": n, "chunk_bytes": seg, "chunks": nseg, "compressed_bytes": enc.total, "ratio": round(enc.total / n, 5),
        "compress_GBps": round(n / min(tc) / 1e9, 2), "decompress_GBps": round(n / min(td) / 1e9, 2),
        "compress_ms": round(1e3 * min(tc), 2), "decompress_ms": round(1e3 * min(td), 2),
        "pinned_h2d_GBps": round(rates["h2d"], 2), "pinned_d2h_GBps": round(rates["d2h"], 2),
        "note": "wall clock, inputs and outputs in pinned host memory, every host<->device copy included; best of "
                f"{reps}",
    }


def selfsync_bench(w, hc, torch, np, indexed_ms: float, reps: int = 5):
    """The workload's streams decoded without their sub-block index, each
    form one batched call over all segments: hc_decode_batch_selfsync (each
    block's pieces resynchronised on the code boundaries, one work-group per
    block) against hc_decode_batch with S = 0 (one lane per block, the
    paper's own decomposition) on the same streams, and the indexed decode
    of the timed step.  Every output is checked against the input; HIP
    events over 'reps' calls of each."""
    items = hc.make_items(w.nseg)
    for t in range(w.nseg):
        hc.set_item(items, t, x=w.outs(t), n=w.seg, in_bytes=w.C[t], dcb=w.dcb[t], out=w.ys(t), block_off=w.off[t])
    ws = torch.empty(max(hc.hc_batch_workspace_bytes(items, w.B), 256), dtype=torch.uint8, device="cuda")
    forms = {
        "selfsync_batched": lambda: hc.hc_decode_batch_selfsync(items, w.B, ws, w.err),
        "lane_per_block_batched": lambda: hc.hc_decode_batch(items, w.B, 0, ws, w.err),
    }
    E = torch.cuda.Event
    out = {}
    for name, fn in forms.items():
        w.y.zero_()
        fn()
        torch.cuda.synchronize()
        if hc.read_error(w.err):
            raise hc.HcError(hc.read_error(w.err), name)
        assert torch.equal(w.y, w.x), f"{name}: round trip failed"
        s, e = E(enable_timing=True), E(enable_timing=True)
        s.record()
        for _ in range(reps):
            fn()
        e.record()
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / reps
        out[name] = {"ms": round(ms, 3), "GBps": round(w.n / ms / 1e6, 1)}
    if hc.read_error(w.err):
        raise hc.HcError(hc.read_error(w.err), "index-free decodes (timed)")
    assert torch.equal(w.y, w.x), "index-free decodes: round trip failed (timed)"
    out["indexed_batched"] = {"ms": round(indexed_ms, 3), "GBps": round(w.n / indexed_ms / 1e6, 1),
                              "sub_block": w.S}
    out.update({"block_size": w.B, "streams": w.nseg,
                "note": "each form one batched call over every segment, HIP events over "
                        f"{reps} calls; GBps of decoded bytes"})
    return out


def copy_probe(hc, torch, quiet=False):
    """The library's roofline probes over 1 GiB: a streaming device copy
    (read + write) and a streaming read.  Returns both rates in GB/s; the
    copy is the achievable side of the codec kernels' roofline."""
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    a.fill_(1)
    E = torch.cuda.Event
    reps = 20
    ms = {}
    for name, fn in (("copy", lambda: hc.hc_probe_copy(a, b)), ("read", lambda: hc.hc_probe_read(a, sink))):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        s, e = E(enable_timing=True), E(enable_timing=True)
        s.record()
        for _ in range(reps):
            fn()
        e.record()
        torch.cuda.synchronize()
        ms[name] = s.elapsed_time(e) / reps
    del a, b
    copy_rate, read_rate = 2 * n / ms["copy"] / 1e6, n / ms["read"] / 1e6
    if not quiet:
        print(json.dumps({"probe": "hc_probe_copy / hc_probe_read", "bytes": n, "copy_ms": round(ms["copy"], 4),
                          "copy_GBps_read_plus_write": round(copy_rate, 1), "read_ms": round(ms["read"], 4),
                          "read_GBps": round(read_rate, 1)}), flush=True)
    return copy_rate, read_rate


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the codec has no multi-GPU path (its independent streams "
              "would shard across GPUs with no exchange).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1107_1525_amd as hc
    import synth

    # the timed run tunes its launch parameters unless any of them is given
    # (the helper modes take the defaults)
    tune_wanted = (args.block is None and args.sub_block is None and args.tile_loads is None and not args.no_tune
                   and not (args.sweep or args.per_kind or args.traffic_summary or args.sq_table or args.trace_summary
                            or args.copy_probe))

    def fill_defaults():
        args.block = 64 * 1024 if args.block is None else args.block
        args.sub_block = 128 if args.sub_block is None else args.sub_block
        args.tile_loads = 0 if args.tile_loads is None else args.tile_loads

    if not tune_wanted:
        fill_defaults()
    if args.traffic_summary:
        traffic_summary(args.traffic_summary, args.block, args.sub_block)
        return
    if args.sq_table:
        sq_table(args.sq_table, synth, args)
        return
    if args.trace_summary:
        trace_summary(args.trace_summary, args.block, args.sub_block)
        return
    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe(hc, torch)
        return
    if args.per_kind:
        per_kind_bench(hc, synth, torch, np, args)
        return

    tuned = None
    if tune_wanted:
        print(f"[bench] autotuning on {args.tune_segments} x 64 MiB", file=sys.stderr, flush=True)
        tuned = autotune_step(hc, synth, torch, args.tune_segments)
        args.block, args.sub_block = tuned["best"]["block_size"], tuned["best"]["sub_block"]
        args.tile_loads = tuned["best"]["encode_tile_loads"]
        fill_defaults()
    hc.hc_set_tuning(args.tile_loads)
    configs = [(args.block, args.sub_block)]
    if args.sweep:
        configs = [(B, S) for B in (4096, 16384, 65536, 262144) for S in ((0,) if B == 4096 else (0, 512, 1024, 4096))]

    for B, S in configs:
        print(f"[bench] setting up {args.segments} x 64 MiB, B={B} S={S}", file=sys.stderr, flush=True)
        w = Workload(hc, synth, torch, args.segments, B, S)
        w.run(args.warmup)
        torch.cuda.synchronize()
        if hc.read_error(w.err):
            raise hc.HcError(hc.read_error(w.err), "warmup")
        # correctness of the timed configuration: decode must reproduce the input
        assert torch.equal(w.y, w.x), "round trip failed"
        print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
        # HIP events around every launch of the timed steps, on the stream the
        # library launches on (torch's current stream)
        E = torch.cuda.Event
        evs = [{k: (E(enable_timing=True), E(enable_timing=True)) for k in ("hist", "copy", "enc", "dec")}
               for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        w.run(args.steps, evs)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if hc.read_error(w.err):
            raise hc.HcError(hc.read_error(w.err), "timed steps")
        ms_step = wall * 1e3 / args.steps
        avg = lambda k: float(np.mean([e[k][0].elapsed_time(e[k][1]) for e in evs]))
        hist_ms, enc_ms, dec_ms = avg("hist"), avg("enc"), avg("dec")
        # the 2 KiB-per-stream count read-back (GPU time of the copy) and the
        # host code build (host clock), each alone
        readback_ms = float(np.mean([e["hist"][1].elapsed_time(e["copy"][1]) for e in evs]))
        build_ms = 1e3 * float(np.mean([e["host"] for e in evs]))
        copy_rate, read_rate = copy_probe(hc, torch, quiet=True)
        kt = kernel_times(w, torch, np)
        if hc.read_error(w.err):
            raise hc.HcError(hc.read_error(w.err), "kernel timing")
        assert torch.equal(w.y, w.x), "round trip failed (kernel timing)"
        n = w.n
        C = sum(w.C)
        off_bytes = 8 * (w.nb + 1) * w.nseg
        sub_bytes = 4 * w.nsub * w.nseg
        gb = lambda nbytes, ms: nbytes / (ms * 1e-3) / 1e9
        # algorithmic bytes per launch: what each step must move (scratch of the
        # implementation, such as per-tile counts, is not counted)
        # the length pass need not read a stream whose code is a complete
        # 8-bit code (every symbol costs 8 bits): only the other streams count
        complete8 = [bool(np.all(np.asarray(d.host.lengths) == 8)) for d in w.dcb]
        count_bytes = w.seg * sum(1 for c in complete8 if not c)
        alg = {
            "k_hist": n + 8 * 256 * w.nseg,
            "k_count": count_bytes,
            "k_offsets": off_bytes,
            "k_encode": n + C + off_bytes + sub_bytes,
            "k_decode": C + n + off_bytes + sub_bytes,
        }
        kinds = None if args.only_step else kind_kernel_times(w, synth, torch, np)
        if hc.read_error(w.err):
            raise hc.HcError(hc.read_error(w.err), "per-kind timing")
        assert torch.equal(w.y, w.x), "round trip failed (per-kind timing)"
        kavg = {k: float(np.mean(v)) for k, v in kt.items()}
        kernels = {
            k: {"avg_ms": round(kavg[k], 4), "p10_ms": round(float(np.percentile(kt[k], 10)), 4),
                "p50_ms": round(float(np.percentile(kt[k], 50)), 4), "p90_ms": round(float(np.percentile(kt[k], 90)), 4),
                "GBps_alg": round(gb(alg[k], kavg[k]), 1), "pct_hbm": round(100 * gb(alg[k], kavg[k]) / HBM_PEAK_GBPS, 1)}
            for k in KERNELS
        }
        phases = {
            "hist_GBps": round(gb(n, hist_ms), 1),
            "encode_GBps": round(gb(n, enc_ms), 1),
            "decode_GBps": round(gb(n, dec_ms), 1),
            "compress_GBps": round(gb(n, hist_ms + enc_ms), 1),
            "hist_ms": round(hist_ms, 3), "encode_ms": round(enc_ms, 3), "decode_ms": round(dec_ms, 3),
            "encode_pct_hbm": round(100 * gb(n + C + off_bytes + sub_bytes, enc_ms) / HBM_PEAK_GBPS, 1),
            "decode_pct_hbm": round(100 * gb(alg["k_decode"], dec_ms) / HBM_PEAK_GBPS, 1),
            "ratio": round(C / n, 5),
            "count_readback_ms": round(readback_ms, 3), "host_code_build_ms": round(build_ms, 3),
        }
        # the encode and decode calls launch each code class apart, side by
        # side (complete 8-bit codes by the copy forms, the rest by the length
        # pass, the packing and the table decoder), so k_encode and k_decode
        # above are calls; their launches are timed here one at a time, on
        # the segments each serves
        classes = class_launch_times(w, torch, np)
        if hc.read_error(w.err):
            raise hc.HcError(hc.read_error(w.err), "launch-class timing")
        assert torch.equal(w.y, w.x), "round trip failed (launch-class timing)"
        for name, cls, step in (("k_encode_copy", "copy", "k_encode"), ("k_decode_copy", "copy", "k_decode"),
                                ("k_encode_pack", "table", "k_encode"), ("k_decode_table", "table", "k_decode")):
            if cls in classes:
                c = classes[cls]
                ms, nbytes = c["ms"][step], c["alg"][step]
                alg[name] = nbytes
                kavg[name] = ms
                kernels[name] = {"avg_ms": round(ms, 4), "GBps_alg": round(gb(nbytes, ms), 1),
                                 "pct_hbm": round(100 * gb(nbytes, ms) / HBM_PEAK_GBPS, 1),
                                 "note": f"one launch: {c['segments']} segments ({cls} class) alone"}
        # single launches only (a call's launches overlap; the offset pass is
        # one launch per class and too short to matter)
        single = [k for k in ("k_hist", "k_count", "k_encode_copy", "k_encode_pack", "k_decode_copy",
                              "k_decode_table") if k in kavg]
        dominant = max(single, key=lambda k: kavg[k])
        staged = 0 < S <= 128  # the table decoder is k_decode_stage; else a k_decode_ring instance beside the copy's
        symbol = KERNEL_SYMBOL[dominant] if (dominant != "k_decode_table" or staged) else "k_decode_ring"
        one_instance = dominant in SINGLE_INSTANCE and (dominant != "k_decode_table" or staged)
        for k, what in (("k_encode", "encode"), ("k_decode", "decode")):
            kernels[k]["note"] = f"the {what} call: its class launches side by side"
        launch_ms, per_launch = kavg[dominant], alg[dominant]
        achieved = per_launch / (launch_ms * 1e-3) / 1e9
        roofline = {
            "bound": "hbm", "kernel": symbol, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": load_traffic(symbol, B, S) if one_instance else None,
            "launch": dominant,
            "bytes_per_launch": int(per_launch), "launch_ms": round(launch_ms, 4),
            # what the library's streaming copy probe reaches on this device
            # (1 GiB, read + write), and its streaming read alone
            "achievable": round(copy_rate, 1), "frac_of_achievable": round(achieved / copy_rate, 4),
            "achievable_read": round(read_rate, 1),
        }
        line = {
            "metric": METRIC, "value": round(gb(n, ms_step), 2), "unit": "GB/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
            "config": {"workload": WORKLOAD, "bytes": n, "segments": w.nseg, "block_size": B, "sub_block": S,
                       "encode_tile_loads": args.tile_loads,
                       "parallelism": "single-gpu"},
            "phases": phases, "kernels": kernels, "roofline": roofline, "kinds": kinds,
        }
        if tuned is not None:
            line["autotune"] = tuned
        if args.only_step:
            args.no_selfsync = args.no_cpu_baseline = True
            args.batched = args.serve = 0
            args.host_pipeline = False
        if not args.no_selfsync:
            print("[bench] decode without the sub-block index", file=sys.stderr, flush=True)
            line["selfsync_decode"] = selfsync_bench(w, hc, torch, np, kavg["k_decode"])
        if not args.no_cpu_baseline and not args.sweep:
            print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
            line["cpu_baseline"] = cpu_baseline(w, __import__("oracle"), np)
        del w
        torch.cuda.empty_cache()
        if not args.sweep and not args.only_step:
            print("[bench] single streams: 1 MiB and 256 MiB", file=sys.stderr, flush=True)
            line["single_stream"] = [single_stream_bench(hc, synth, torch, np, nm, S)
                                     for nm in ("zipf1.2-1MiB-B4KiB", "zipf1.1-256MiB-B64KiB")]
            torch.cuda.empty_cache()
        if args.batched:
            print(f"[bench] batched: {args.batched} buffers", file=sys.stderr, flush=True)
            line["batched"] = batched_bench(hc, synth, torch, np, args.batched, B, S)
            torch.cuda.empty_cache()
        if args.host_pipeline:
            print("[bench] host-resident pipeline", file=sys.stderr, flush=True)
            line["host_pipeline"] = host_pipeline_bench(hc, synth, torch, np, args.segments, B, S)
            torch.cuda.empty_cache()
        if args.serve:
            print(f"[bench] serving: {args.serve} requests", file=sys.stderr, flush=True)
            line["serving"] = serve_bench(hc, synth, torch, np, args.serve, B, S)
            torch.cuda.empty_cache()
        print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
