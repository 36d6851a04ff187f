"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Integer work, so the bar is bit-exact equality of histograms, code lengths,
code values, block bit counts, offsets, sub-block index, stream bytes and
decoded bytes.  Full-size workloads are checked on sampled blocks (each block
is an independent encoding, so the oracle can encode a sampled block alone)
plus properties that hold at any size (round trip, size = sum of block sizes).
"""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

KIB, MIB = synth.KIB, synth.MIB


@pytest.fixture(scope="module")
def hc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1107_1525_amd as hc_mod

    return hc_mod


def dev(x: np.ndarray) -> torch.Tensor:
    t = torch.empty(max(x.size, 16), dtype=torch.uint8, device="cuda")[: x.size]
    t.copy_(torch.from_numpy(np.ascontiguousarray(x)))
    return t


def u64(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def u32(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def check_full(hc, oracle, x: np.ndarray, B: int, S: int = 0, tag: str = ""):
    """Every output against the oracle, element by element."""
    print(f"[parity] {tag} n={x.size} B={B} S={S}", flush=True)
    xd = dev(x)
    h_gpu = u64(hc.hc_histogram(xd))
    h_or = oracle.histogram(x)
    assert np.array_equal(h_gpu, h_or)
    cb = hc.hc_build_codebook(h_gpu)
    L, C = oracle.codebook(h_or)
    assert np.array_equal(cb.lengths, L) and np.array_equal(cb.codes, C)
    enc = hc.compress(xd, B, sub_block=S, codebook=hc.DeviceCodebook(cb))
    s_or, off_or, bits_or = oracle.encode(x, B, L, C)
    assert np.array_equal(u64(enc.block_off), off_or)
    assert enc.nbytes == s_or.size
    assert np.array_equal(enc.stream.cpu().numpy(), s_or)
    if S:
        assert np.array_equal(u32(enc.sub_idx)[: hc.hc_sub_index_entries(x.size, B, S)],
                              oracle.sub_index(x, B, S, L))
    y = hc.decompress(enc)
    assert torch.equal(y, xd)
    y2 = hc.decompress(enc, use_offsets=False)  # offsets rebuilt by walking the headers
    assert torch.equal(y2, xd)
    return enc


# ------------------------------------------------------------------ histogram
@pytest.mark.parametrize("n", [0, 1, 15, 16, 17, 4095, 131072 + 5, (1 << 20) + 7, 3 * MIB + 1])
@pytest.mark.parametrize("kind", ["zipf", "uniform", "skewed", "const"])
def test_histogram(hc, oracle, n, kind):
    if kind == "zipf":
        x = synth.zipf_bytes(n, 1.2, n + 1)
    elif kind == "uniform":
        x = synth.uniform_bytes(n, n + 2)
    elif kind == "skewed":
        x = synth.skewed_bytes(n, n + 3)
    else:
        x = np.full(n, 0xA5, np.uint8)
    assert np.array_equal(u64(hc.hc_histogram(dev(x))), oracle.histogram(x))


# ------------------------------------------------------------------ small full parity
def test_small_workload_1mib(hc, oracle):
    spec = synth.WORKLOADS["zipf1.2-1MiB-B4KiB"]
    x = synth.zipf_bytes(spec["n"], spec["s"], synth.derive_seed(spec["config_id"], 0))
    check_full(hc, oracle, x, spec["block"], 0, "1MiB zipf1.2 B=4KiB")
    check_full(hc, oracle, x, spec["block"], 1024, "1MiB zipf1.2 B=4KiB S=1KiB")


@pytest.mark.parametrize("B,S", [(16, 0), (48, 16), (4096, 256), (4112, 0), (6016, 512), (16384, 1024),
                                 (65536, 4096), (262144, 0), (1 << 20, 65536),
                                 # encode tiles of 2 and 4 loads per thread, index entries on every load
                                 (8192, 16), (8208, 16), (16384, 16), (65536, 48), (32768 + 4096, 32)])
def test_block_sizes(hc, oracle, B, S):
    x = synth.zipf_bytes(2 * MIB + 333, 1.1, B)
    check_full(hc, oracle, x, B, S, "zipf1.1 ragged")


@pytest.mark.parametrize("kind", ["zipf", "uniform", "skewed"])
@pytest.mark.parametrize("shift_in,shift_out", [(16, 0), (48, 32), (112, 80), (64, 112)])
def test_decode_unaligned_lines(hc, oracle, kind, shift_in, shift_out):
    """Stream and output 16-byte aligned but not at the start of a 128-byte
    line: the decoder's line-wide loads and stores must touch only the chunk's
    own bytes (neighbouring bytes keep a sentinel)."""
    x = (synth.zipf_bytes(300_000 + 13, 1.2, 5) if kind == "zipf" else synth.segment_bytes(kind, 300_000 + 13, 5))
    B, S = 16384, 1024
    enc = check_full(hc, oracle, x, B, S, f"{kind} unaligned {shift_in}/{shift_out}")
    sbuf = torch.full((enc.nbytes + 256,), 0xA5, dtype=torch.uint8, device="cuda")
    sbuf[shift_in:shift_in + enc.nbytes].copy_(enc.stream[: enc.nbytes])
    obuf = torch.full((x.size + 256,), 0x5A, dtype=torch.uint8, device="cuda")
    err = hc.new_error_word("cuda")
    hc.hc_decode_blocks(sbuf[shift_in:], enc.nbytes, x.size, B, enc.codebook, enc.block_off, enc.sub_idx, S,
                        obuf[shift_out:], err)
    assert hc.read_error(err) == 0
    o = obuf.cpu().numpy()
    assert np.array_equal(o[shift_out:shift_out + x.size], x)
    assert (o[:shift_out] == 0x5A).all() and (o[shift_out + x.size:] == 0x5A).all()


@pytest.mark.parametrize("n", [1, 15, 16, 17, 4095, 4096, 4097, 8191, 8193, 65535, 65536, 65537])
def test_ragged_sizes(hc, oracle, n):
    x = synth.zipf_bytes(n, 1.3, 7 * n)
    check_full(hc, oracle, x, 4096, 0, "ragged")
    check_full(hc, oracle, x, 65536, 1024, "ragged multi-tile")


@pytest.mark.parametrize("kind", ["uniform", "skewed", "fp32"])
def test_segment_kinds(hc, oracle, kind):
    x = synth.segment_bytes(kind, 3 * MIB, 11)
    for B in (4 * KIB, 16 * KIB, 64 * KIB, 256 * KIB):
        check_full(hc, oracle, x, B, 1024 if B > 4 * KIB else 0, kind)


def test_single_symbol(hc, oracle):
    x = np.full(100_000, 42, np.uint8)
    enc = check_full(hc, oracle, x, 4096, 512, "single symbol")
    assert enc.codebook.max_len == 1


def test_all_symbols_equal_counts(hc, oracle):
    x = np.tile(np.arange(256, dtype=np.uint8), 4096)
    np.random.default_rng(1).shuffle(x)
    check_full(hc, oracle, x, 16384, 1024, "all 256 symbols")


def _codebook_from_counts(hc, oracle, counts):
    h = np.zeros(256, np.uint64)
    h[: len(counts)] = counts
    cb = hc.hc_build_codebook(h)
    L, C = oracle.codebook(h)
    assert np.array_equal(cb.lengths, L) and np.array_equal(cb.codes, C)
    return cb, L, C


@pytest.mark.parametrize("m", [14, 20, 26, 33, 45, 65])
def test_long_codes(hc, oracle, m):
    """Fibonacci counts give codes of m-1 bits: the LUT fallback (>12 bits),
    the 24-bit packed table limit and the 64-bit general path."""
    fib = [1, 1]
    while len(fib) < m:
        fib.append(fib[-1] + fib[-2])
    cb, L, C = _codebook_from_counts(hc, oracle, fib)
    assert cb.max_len == m - 1
    rng = np.random.default_rng(m)
    x = rng.integers(0, m, size=300_001).astype(np.uint8)  # every symbol, long codes frequent
    xd = dev(x)
    for B, S in ((4096, 0), (16384, 1024), (65536, 4096)):
        enc = hc.compress(xd, B, sub_block=S, codebook=hc.DeviceCodebook(cb))
        s_or, off_or, _ = oracle.encode(x, B, L, C)
        assert np.array_equal(u64(enc.block_off), off_or)
        assert np.array_equal(enc.stream.cpu().numpy(), s_or)
        if S:
            assert np.array_equal(u32(enc.sub_idx), oracle.sub_index(x, B, S, L))
        assert torch.equal(hc.decompress(enc), xd)


def test_determinism(hc, oracle):
    x = synth.skewed_bytes(5 * MIB + 3, 5)
    xd = dev(x)
    a = hc.compress(xd, 16384, sub_block=1024)
    b = hc.compress(xd, 16384, sub_block=1024)
    assert torch.equal(a.stream, b.stream) and torch.equal(a.block_off, b.block_off)
    assert torch.equal(a.sub_idx, b.sub_idx)


# ------------------------------------------------------------------ errors
def test_symbol_absent(hc, oracle):
    L = np.zeros(256, np.uint8)
    L[[1, 2]] = 1
    cb = hc.DeviceCodebook(hc.hc_codebook_from_lengths(L))
    with pytest.raises(hc.HcError) as e:
        hc.compress(dev(np.array([1, 2, 3] * 100, np.uint8)), 64, codebook=cb)
    assert e.value.status == hc.HC_ERR_SYMBOL_ABSENT


def _decode_status(hc, stream_np, enc, n=None, sub=True):
    err = hc.new_error_word("cuda")
    s = dev(stream_np)
    n = enc.n if n is None else n
    out = torch.empty(max(n, 16), dtype=torch.uint8, device="cuda")
    nb = hc.num_blocks(n, enc.block_size)
    off = torch.zeros(nb + 1, dtype=torch.int64, device="cuda")
    hc.hc_walk_blocks(s, s.numel(), nb, off, err)
    if hc.read_error(err):
        return hc.read_error(err)
    use_sub = sub and enc.sub_idx is not None and n == enc.n
    hc.hc_decode_blocks(s, s.numel(), n, enc.block_size, enc.codebook, off,
                        enc.sub_idx if use_sub else None, enc.sub_block if use_sub else 0, out, err)
    return hc.read_error(err)


@pytest.mark.parametrize("kind", ["zipf", "skewed"])
def test_corruption_matches_oracle(hc, oracle, kind):
    x = synth.zipf_bytes(200_000, 1.2, 1) if kind == "zipf" else synth.skewed_bytes(200_000, 1)
    B = 4096
    enc = hc.compress(dev(x), B, sub_block=1024)
    L = enc.codebook.host.lengths
    s0 = enc.stream.cpu().numpy()
    off = u64(enc.block_off)
    bits = np.array([int.from_bytes(s0[int(o):int(o) + 4].tobytes(), "little") for o in off[:-1]])
    assert _decode_status(hc, s0, enc) == 0 and oracle.decode_status(s0, x.size, B, L)[0] == 0
    cases = {}
    s = s0.copy(); s[int(off[5])] ^= 1; cases["header bit"] = s
    s = s0.copy(); s[int(off[-2]) + 3] = 0x7F; cases["header too large"] = s
    i = next(i for i in range(bits.size) if bits[i] % 32)
    pb = int(bits[i]); w = int(off[i]) + 4 + 4 * (pb // 32); pos = 31 - pb % 32
    s = s0.copy(); s[w + pos // 8] |= 1 << (pos % 8); cases["nonzero pad"] = s
    cases["truncated"] = s0[:-4].copy()
    cases["trailing"] = np.concatenate([s0, np.zeros(4, np.uint8)])
    for name, s in cases.items():
        st_or = oracle.decode_status(s, x.size, B, L)[0]
        st_gpu = _decode_status(hc, s, enc)
        assert st_or == oracle.ERR_CORRUPT, name
        assert st_gpu == hc.HC_ERR_CORRUPT, name
    # wrong symbol count
    assert _decode_status(hc, s0, enc, n=x.size + B, sub=False) == hc.HC_ERR_CORRUPT
    # a sub-block index that disagrees with the stream
    bad = enc.sub_idx.clone()
    bad[1] += 1
    err = hc.new_error_word("cuda")
    out = torch.empty(x.size, dtype=torch.uint8, device="cuda")
    hc.hc_decode_blocks(enc.stream, enc.nbytes, enc.n, B, enc.codebook, enc.block_off, bad, 1024, out, err)
    assert hc.read_error(err) == hc.HC_ERR_CORRUPT


def test_invalid_code_foreign_codebook(hc, oracle):
    L = np.zeros(256, np.uint8)
    L[[1, 2]] = [1, 2]  # "11" is no code
    cb = hc.DeviceCodebook(hc.hc_codebook_from_lengths(L))
    x = np.array([1, 2, 1, 1] * 8, np.uint8)
    enc = hc.compress(dev(x), 16, codebook=cb)
    s = enc.stream.cpu().numpy().copy()
    s[4 + 3] |= 0xC0
    assert oracle.decode_status(s, x.size, 16, L)[0] == oracle.ERR_CORRUPT
    assert _decode_status(hc, s, enc, sub=False) == hc.HC_ERR_CORRUPT


# ------------------------------------------------------------------ full-size workloads, sampled
def _sampled_blocks(hc, oracle, x_dev, enc, L, C, nsample, rng):
    n, B = enc.n, enc.block_size
    nb = hc.num_blocks(n, B)
    off = u64(enc.block_off)
    picks = sorted(set([0, nb - 1] + rng.integers(0, nb, size=nsample).tolist()))
    for i in picks:
        a = i * B
        blk = x_dev[a:a + B].cpu().numpy()
        s_or, off_or, _ = oracle.encode(blk, B, L, C)
        got = enc.stream[int(off[i]):int(off[i + 1])].cpu().numpy()
        assert np.array_equal(got, s_or), f"block {i}"
        if enc.sub_idx is not None:
            cpb = (B + enc.sub_block - 1) // enc.sub_block
            assert np.array_equal(u32(enc.sub_idx[i * cpb:(i + 1) * cpb]),
                                  oracle.sub_index(blk, B, enc.sub_block, L)), f"index {i}"


def test_single_stream_256mib(hc, oracle):
    spec = synth.WORKLOADS["zipf1.1-256MiB-B64KiB"]
    n, B = spec["n"], spec["block"]
    print(f"[parity] 256MiB zipf1.1 B=64KiB", flush=True)
    x = synth.zipf_bytes_torch(n, spec["s"], synth.derive_seed(spec["config_id"], 0))
    h = u64(hc.hc_histogram(x))
    x_host = x.cpu().numpy()
    assert np.array_equal(h, oracle.histogram(x_host))
    cb = hc.hc_build_codebook(h)
    L, C = oracle.codebook(h)
    assert np.array_equal(cb.lengths, L) and np.array_equal(cb.codes, C)
    enc = hc.compress(x, B, sub_block=1024, codebook=hc.DeviceCodebook(cb))
    bits_or = oracle.block_bits(x_host, B, L)
    off_or = np.concatenate([[0], np.cumsum(4 + 4 * ((bits_or + 31) // 32))]).astype(np.uint64)
    assert np.array_equal(u64(enc.block_off), off_or)
    _sampled_blocks(hc, oracle, x, enc, L, C, 24, np.random.default_rng(2))
    assert torch.equal(hc.decompress(enc), x)


def test_mixed_4gib_sampled(hc, oracle):
    """The 4 GiB mixed workload: 64 segments of 64 MiB with their own codebooks,
    at every block size the benchmark sweeps, with the launch shapes it uses."""
    spec = synth.WORKLOADS["mixed-4GiB-64x64MiB"]
    seg = spec["segment"]
    nseg = spec["n"] // seg
    rng = np.random.default_rng(3)
    x = torch.empty(spec["n"], dtype=torch.uint8, device="cuda")
    for t in range(nseg):
        synth.segment_bytes_torch(synth.mixed_kind(t), seg, synth.derive_seed(spec["config_id"], t),
                                  out=x[t * seg:(t + 1) * seg])
    checked = {0, 1, 2, nseg - 1}
    for t in range(nseg):
        xs = x[t * seg:(t + 1) * seg]
        h = u64(hc.hc_histogram(xs))
        assert int(h.sum()) == seg
        if t in checked:
            print(f"[parity] 4GiB segment {t} ({synth.mixed_kind(t)})", flush=True)
            assert np.array_equal(h, oracle.histogram(xs.cpu().numpy()))
            cb = hc.hc_build_codebook(h)
            L, C = oracle.codebook(h)
            assert np.array_equal(cb.lengths, L) and np.array_equal(cb.codes, C)
            dcb = hc.DeviceCodebook(cb)
            for B in spec["blocks"]:
                enc = hc.compress(xs, B, sub_block=1024 if B > 4 * KIB else 0, codebook=dcb)
                _sampled_blocks(hc, oracle, xs, enc, L, C, 4, rng)
                assert torch.equal(hc.decompress(enc), xs)
    del x
    torch.cuda.empty_cache()


def test_codebook_update_in_place(hc, oracle):
    """hc_codebook_update swaps the tables of a handle on the stream: work
    enqueued before sees the old code, work enqueued after the new one."""
    xa = synth.zipf_bytes(300_000, 1.2, 21)
    xb = synth.skewed_bytes(300_000, 22)
    La, Ca = oracle.codebook(oracle.histogram(xa))
    Lb, Cb = oracle.codebook(oracle.histogram(xb))
    dcb = hc.DeviceCodebook(hc.hc_build_codebook(oracle.histogram(xa)))
    enc_a = hc.compress(dev(xa), 4096, codebook=dcb, check=False)
    dcb.update(hc.hc_build_codebook(oracle.histogram(xb)))
    enc_b = hc.compress(dev(xb), 4096, codebook=dcb)
    assert np.array_equal(enc_a.stream.cpu().numpy(), oracle.encode(xa, 4096, La, Ca)[0])
    assert np.array_equal(enc_b.stream.cpu().numpy(), oracle.encode(xb, 4096, Lb, Cb)[0])
    assert torch.equal(hc.decompress(enc_b), dev(xb))
    for _ in range(3):  # repeated updates reuse the staging area
        dcb.update(hc.hc_build_codebook(oracle.histogram(xa)))
        dcb.update(hc.hc_build_codebook(oracle.histogram(xb)))
    enc_b2 = hc.compress(dev(xb), 4096, codebook=dcb)
    assert torch.equal(enc_b2.stream, enc_b.stream)


def test_walk_matches_encoder_offsets(hc, oracle):
    x = synth.zipf_bytes(1_000_003, 1.1, 23)
    enc = hc.compress(dev(x), 4096)
    nb = hc.num_blocks(x.size, 4096)
    off = torch.zeros(nb + 1, dtype=torch.int64, device="cuda")
    err = hc.new_error_word("cuda")
    hc.hc_walk_blocks(enc.stream, enc.nbytes, nb, off, err)
    assert hc.read_error(err) == 0
    assert torch.equal(off, enc.block_off)
    assert np.array_equal(u64(off), oracle.walk(enc.stream.cpu().numpy(), nb))


# ------------------------------------------------------------------ batches
@pytest.mark.parametrize("B,S", [(4096, 0), (65536, 1024), (16384, 512)])
def test_batch_matches_single_and_oracle(hc, oracle, B, S):
    """Buffers of uneven sizes (empty and tiny included), each with its own
    codebook, in one launch per step: every result equals the single-buffer
    call and the oracle."""
    rng = np.random.default_rng(B + S)
    sizes = [0, 1, 17, 4096, 70_001, 333_333, 1 << 20, 5]
    kinds = ["zipf", "uniform", "skewed", "fp32"]
    xs = []
    for k, n in enumerate(sizes):
        kind = kinds[k % 4]
        if kind == "zipf":
            xs.append(synth.zipf_bytes(n, float(rng.uniform(0.8, 1.6)), k))
        elif kind == "fp32":
            xs.append(synth.fp32_bytes((n + 3) // 4 * 4, k)[:n])
        else:
            xs.append(synth.segment_bytes(kind, n, k))
    xd = [dev(x) for x in xs]
    cnt = len(xs)
    items = hc.make_items(cnt)
    hists = [torch.empty(256, dtype=torch.int64, device="cuda") for _ in xs]
    for k in range(cnt):
        hc.set_item(items, k, x=xd[k], hist=hists[k])
    ws = torch.empty(max(hc.hc_batch_workspace_bytes(items, B), 256), dtype=torch.uint8, device="cuda")
    hc.hc_histogram_batch(items, ws)
    dcbs, outs, offs, subs = [], [], [], []
    for k in range(cnt):
        h = u64(hists[k])
        assert np.array_equal(h, oracle.histogram(xs[k])), k
        cb = hc.hc_build_codebook(h)
        if cb.max_len == 0:
            L0 = np.zeros(256, np.uint8)
            L0[0] = 1
            cb = hc.hc_codebook_from_lengths(L0)
        dcbs.append(hc.DeviceCodebook(cb))
        n = xs[k].size
        outs.append(torch.empty(max(hc.hc_encode_bound(n, B, cb.max_len), 16), dtype=torch.uint8, device="cuda"))
        offs.append(torch.empty(hc.num_blocks(n, B) + 1, dtype=torch.int64, device="cuda"))
        subs.append(torch.empty(max(hc.hc_sub_index_entries(n, B, S), 1), dtype=torch.int32, device="cuda")
                    if S else None)
        hc.set_item(items, k, x=xd[k], dcb=dcbs[k], out=outs[k], block_off=offs[k], sub_idx=subs[k])
    ws = torch.empty(max(hc.hc_batch_workspace_bytes(items, B), 256), dtype=torch.uint8, device="cuda")
    err = hc.new_error_word("cuda")
    hc.hc_encode_batch(items, B, S, ws, err)
    assert hc.read_error(err) == 0
    # the three step calls give the same bytes as the one-call encode
    whole = [(o.clone(), f.clone(), None if u is None else u.clone()) for o, f, u in zip(outs, offs, subs)]
    for o, f, u in zip(outs, offs, subs):
        o.fill_(0x5A)
        f.fill_(-1)
        if u is not None:
            u.fill_(-1)
    hc.hc_encode_lengths_batch(items, B, S, ws, err)
    hc.hc_encode_offsets_batch(items, B, S, ws, err)
    hc.hc_encode_pack_batch(items, B, S, ws, err)
    assert hc.read_error(err) == 0
    for k in range(cnt):
        C = int(whole[k][1][-1].item())
        assert torch.equal(outs[k][:C], whole[k][0][:C]), k
        assert torch.equal(offs[k], whole[k][1]), k
        if S:
            m = hc.hc_sub_index_entries(xs[k].size, B, S)
            assert torch.equal(subs[k][:m], whole[k][2][:m]), k
    ys = []
    for k in range(cnt):
        n = xs[k].size
        C = int(offs[k][-1].item())
        single = hc.compress(xd[k], B, sub_block=S, codebook=dcbs[k])
        assert torch.equal(outs[k][:C], single.stream), k
        assert torch.equal(offs[k], single.block_off), k
        if S:
            m = hc.hc_sub_index_entries(n, B, S)
            assert torch.equal(subs[k][:m], single.sub_idx[:m]), k
        if n:
            L = dcbs[k].host.lengths
            s_or, off_or, _ = oracle.encode(xs[k], B, L, oracle.canonical_codes(L))
            assert np.array_equal(outs[k][:C].cpu().numpy(), s_or), k
        ys.append(torch.empty(max(n, 16), dtype=torch.uint8, device="cuda"))
        hc.set_item(items, k, x=outs[k], n=n, in_bytes=C, dcb=dcbs[k], out=ys[k], block_off=offs[k], sub_idx=subs[k])
    hc.hc_decode_batch(items, B, S, ws, err)
    assert hc.read_error(err) == 0
    for k in range(cnt):
        assert torch.equal(ys[k][: xs[k].size], xd[k]), k


def test_fixed_length_codes(hc, oracle):
    """All codes 8 bits long (uniform bytes): the decoder's fixed-length path,
    with and without the sub-block index, and its strict checks."""
    x = synth.uniform_bytes(1_000_001, 31)
    for B, S in ((4096, 0), (65536, 1024), (16384, 0)):
        enc = check_full(hc, oracle, x, B, S, "fixed 8-bit codes")
        assert enc.codebook.max_len == 8
    # an incomplete 8-bit code: 200 symbols, bytes >= 200 have no code
    L = np.zeros(256, np.uint8)
    L[:200] = 8
    cb = hc.DeviceCodebook(hc.hc_codebook_from_lengths(L))
    y = (np.arange(50_000) % 200).astype(np.uint8)
    enc = hc.compress(dev(y), 4096, codebook=cb)
    assert torch.equal(hc.decompress(enc), dev(y))
    s = enc.stream.cpu().numpy().copy()
    s[4 + 3] = 0xFF  # first code of block 0 becomes 255
    assert oracle.decode_status(s, y.size, 4096, L)[0] == oracle.ERR_CORRUPT
    assert _decode_status(hc, s, enc, sub=False) == hc.HC_ERR_CORRUPT
    s = enc.stream.cpu().numpy().copy()
    s[0] ^= 8  # header no longer 8 bits per symbol
    assert _decode_status(hc, s, enc, sub=False) == hc.HC_ERR_CORRUPT


def test_complete_8bit_code(hc, oracle):
    """Every byte coded with 8 bits (a complete code): the decoder's copy path.
    Any payload byte is a valid code, so a flipped payload byte decodes as
    the oracle decodes it; header, index and pad corruptions are rejected."""
    x = synth.uniform_bytes(70_003, 32)  # n % 4 != 0: pad bits in the last block
    # S = 128 with B >= 8 KiB: waves whose 64 chunks lie in one whole block take
    # the contiguous copy, the others (the ragged last block) the general one
    for B, S in ((4096, 0), (16384, 1024), (65536, 4096), (16384, 128), (65536, 128)):
        enc = check_full(hc, oracle, x, B, S, "complete 8-bit code")
        L = enc.codebook.host.lengths
        assert np.all(L == 8)
        s = enc.stream.cpu().numpy().copy()
        for pos in (4 + 100, 4 + 4 * 1000 + 2, s.size - 5):
            t = s.copy()
            t[pos] ^= 0x5A
            st, ref = oracle.decode_status(t, x.size, B, L)
            assert st == oracle.OK, pos
            y = hc.decompress(hc.Encoded(dev(t), enc.block_off, enc.sub_idx, enc.n, B, S, enc.codebook))
            assert np.array_equal(y.cpu().numpy(), ref[: x.size]), (B, S, pos)
            assert int((y.cpu().numpy() != x).sum()) == 1, (B, S, pos)
        t = s.copy()
        t[0] ^= 1  # a header no longer 8 bits per symbol
        assert oracle.decode_status(t, x.size, B, L)[0] == oracle.ERR_CORRUPT
        assert _decode_status(hc, t, enc, sub=False) == hc.HC_ERR_CORRUPT
        t = s.copy()
        t[s.size - 4] |= 1  # a pad bit of the last word
        assert oracle.decode_status(t, x.size, B, L)[0] == oracle.ERR_CORRUPT
        assert _decode_status(hc, t, enc, sub=False) == hc.HC_ERR_CORRUPT
        if S:
            bad = enc.sub_idx.clone()
            bad[1] += 8  # an index entry off by one symbol
            err = hc.new_error_word("cuda")
            out = torch.empty(x.size + 16, dtype=torch.uint8, device="cuda")
            hc.hc_decode_blocks(enc.stream, enc.nbytes, enc.n, B, enc.codebook, enc.block_off, bad, S, out, err)
            assert hc.read_error(err) == hc.HC_ERR_CORRUPT


def test_codebook_set(hc, oracle):
    """A set of resident tables rebuilt from histograms in one call gives the
    same codes and streams as separate codebooks, rebuild after rebuild."""
    xs = [synth.zipf_bytes(200_000 + 17 * k, 1.0 + 0.2 * k, 40 + k) for k in range(5)]
    xs.append(np.zeros(0, np.uint8))
    cset = hc.CodebookSet(len(xs))
    for rebuild in range(3):
        order = xs if rebuild % 2 == 0 else xs[::-1]
        hists = np.stack([oracle.histogram(x) for x in order])
        books = cset.build(hists)
        for k, x in enumerate(order):
            if x.size == 0:
                assert books[k].max_len == 1
                continue
            L, C = oracle.codebook(hists[k])
            assert np.array_equal(books[k].host.lengths, L) and np.array_equal(books[k].host.codes, C)
            enc = hc.compress(dev(x), 4096, sub_block=1024, codebook=books[k])
            assert np.array_equal(enc.stream.cpu().numpy(), oracle.encode(x, 4096, L, C)[0])
            assert torch.equal(hc.decompress(enc), dev(x))
    cset.close()


@pytest.mark.parametrize("B,S", [(4096, 0), (65536, 1024)])
def test_batch_graph_replays(hc, oracle, B, S):
    """The three batched calls captured once in a HIP graph and replayed: 70
    buffers (job tables of three argument-carrying launches each), outputs
    cleared eagerly between replays, every replay equal to the eager calls
    and to the oracle on sampled buffers."""
    rng = np.random.default_rng(B + S + 1)
    cnt = 70
    sizes = [0, 1, 5] + [int(v) for v in rng.integers(16, 150_000, cnt - 3)]
    kinds = ["zipf", "uniform", "skewed", "fp32"]
    xs = []
    for k, n in enumerate(sizes):
        kind = kinds[k % 4]
        if kind == "zipf":
            xs.append(synth.zipf_bytes(n, float(rng.uniform(0.8, 1.6)), 500 + k))
        elif kind == "fp32":
            xs.append(synth.fp32_bytes((n + 3) // 4 * 4, 500 + k)[:n])
        else:
            xs.append(synth.segment_bytes(kind, n, 500 + k))
    xd = [dev(x) for x in xs]
    hist = torch.zeros((cnt, 256), dtype=torch.int64, device="cuda")
    h_items = hc.make_items(cnt)
    for k in range(cnt):
        hc.set_item(h_items, k, x=xd[k], hist=hist[k])
    hws = torch.empty(max(hc.hc_batch_workspace_bytes(h_items, B), 256), dtype=torch.uint8, device="cuda")
    hc.hc_histogram_batch(h_items, hws)
    dcbs, outs, offs, subs, ys = [], [], [], [], []
    e_items = hc.make_items(cnt)
    for k in range(cnt):
        cb = hc.hc_build_codebook(u64(hist[k]))
        if cb.max_len == 0:
            L0 = np.zeros(256, np.uint8)
            L0[0] = 1
            cb = hc.hc_codebook_from_lengths(L0)
        dcbs.append(hc.DeviceCodebook(cb))
        n = sizes[k]
        outs.append(torch.zeros(max(hc.hc_encode_bound(n, B, cb.max_len), 16), dtype=torch.uint8, device="cuda"))
        offs.append(torch.zeros(hc.num_blocks(n, B) + 1, dtype=torch.int64, device="cuda"))
        subs.append(torch.zeros(max(hc.hc_sub_index_entries(n, B, S), 1), dtype=torch.int32, device="cuda")
                    if S else None)
        ys.append(torch.zeros(max(n, 16), dtype=torch.uint8, device="cuda"))
        hc.set_item(e_items, k, x=xd[k], dcb=dcbs[k], out=outs[k], block_off=offs[k], sub_idx=subs[k])
    ws = torch.empty(max(hc.hc_batch_workspace_bytes(e_items, B), 256), dtype=torch.uint8, device="cuda")
    err = hc.new_error_word("cuda")
    hc.hc_encode_batch(e_items, B, S, ws, err)
    C = [int(o[-1].item()) for o in offs]
    d_items = hc.make_items(cnt)
    for k in range(cnt):
        hc.set_item(d_items, k, x=outs[k], n=sizes[k], in_bytes=C[k], dcb=dcbs[k], out=ys[k], block_off=offs[k],
                    sub_idx=subs[k])
    hc.hc_decode_batch(d_items, B, S, ws, err)
    torch.cuda.synchronize()
    assert hc.read_error(err) == 0
    eager = [(hist[k].clone(), outs[k][: C[k]].clone(), offs[k].clone(), None if S == 0 else subs[k].clone())
             for k in range(cnt)]
    for k in range(cnt):
        assert torch.equal(ys[k][: sizes[k]], xd[k]), k
    for k in range(1, cnt):  # every buffer against the oracle's own code and encoder
        L, Cw = oracle.codebook(oracle.histogram(xs[k]))
        s_o, off_o, _ = oracle.encode(xs[k], B, L, Cw)
        assert np.array_equal(eager[k][1].cpu().numpy(), s_o), k
        assert np.array_equal(u64(eager[k][2]), off_o), k

    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=side):
        hc.hc_histogram_batch(h_items, hws)
        hc.hc_encode_batch(e_items, B, S, ws, err)
        hc.hc_decode_batch(d_items, B, S, ws, err)
    torch.cuda.synchronize()
    for rep in range(3):
        for t in [hist] + outs + offs + ys + [u for u in subs if u is not None]:
            t.zero_()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert hc.read_error(err) == 0, rep
        for k in range(cnt):
            assert torch.equal(hist[k], eager[k][0]), (rep, k)
            assert torch.equal(outs[k][: C[k]], eager[k][1]), (rep, k)
            assert torch.equal(offs[k], eager[k][2]), (rep, k)
            if S:
                assert torch.equal(subs[k], eager[k][3]), (rep, k)
            assert torch.equal(ys[k][: sizes[k]], xd[k]), (rep, k)


def test_batch_decode_mixed_complete_codes(hc, oracle):
    """A batch mixing complete 8-bit codes (large uniform buffers: decoded by
    the copy launch) with other codes (the ring launch): every buffer decodes
    to its input, and its stream is the oracle's."""
    B, S = 65536, 1024
    sizes = [300_000, 1 << 20, 70_001, 2 << 20, 5, 4096 * 3 + 17, 1 << 20]
    xs = [synth.uniform_bytes(n, 100 + k) if k % 2 == 0 else synth.zipf_bytes(n, 1.1, 100 + k)
          for k, n in enumerate(sizes)]
    encs = [hc.compress(dev(x), B, sub_block=S) for x in xs]
    complete = [e.codebook.max_len == 8 and int(e.codebook.host.nsym) == 256 for e in encs]
    assert any(complete) and not all(complete)
    for x, e in zip(xs, encs):
        L, C = oracle.codebook(oracle.histogram(x))
        assert np.array_equal(e.stream.cpu().numpy(), oracle.encode(x, B, L, C)[0])
    items = hc.make_items(len(xs))
    outs = [torch.empty(max(x.size, 16), dtype=torch.uint8, device="cuda")[: x.size] for x in xs]
    for k, (e, o) in enumerate(zip(encs, outs)):
        hc.set_item(items, k, x=e.stream, n=e.n, in_bytes=e.nbytes, dcb=e.codebook, out=o,
                    block_off=e.block_off, sub_idx=e.sub_idx)
    ws = torch.empty(hc.hc_batch_workspace_bytes(items, B), dtype=torch.uint8, device="cuda")
    err = hc.new_error_word("cuda")
    for _ in range(2):  # the workspace's two job tables reused
        for o in outs:
            o.zero_()
        hc.hc_decode_batch(items, B, S, ws, err)
        torch.cuda.synchronize()
        assert hc.read_error(err) == 0
        for x, o in zip(xs, outs):
            assert np.array_equal(o.cpu().numpy(), x)
