"""Block decoding without the sub-block index (hc_decode_blocks_selfsync:
each block's payload cut into pieces decoded in parallel and resynchronised
on the code boundaries).  Its result has a plain definition, the input the
oracle encoded, so every case checks the stream against the oracle's encoder
and the decode against the input, over the code shapes of the indexed
decoder's tests; and it is as strict: every corruption the oracle rejects is
rejected."""
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


def selfsync(hc, s: torch.Tensor, n: int, enc, off: torch.Tensor):
    out = torch.empty(max(n, 16), dtype=torch.uint8, device="cuda")[:n]
    err = hc.new_error_word("cuda")
    hc.hc_decode_blocks_selfsync(s, s.numel(), n, enc.block_size, enc.codebook, off, out, err)
    return out, hc.read_error(err)


def data(kind: str, n: int, seed: int) -> np.ndarray:
    if kind == "zipf":
        return synth.zipf_bytes(n, 1.2, seed)
    if kind == "const":
        return np.full(n, 7, np.uint8)
    return synth.segment_bytes(kind, n, seed)


def check(hc, oracle, x: np.ndarray, B: int, cb=None, tag=""):
    print(f"[selfsync] {tag} n={x.size} B={B}", flush=True)
    xd = dev(x)
    enc = hc.compress(xd, B, codebook=cb)
    if cb is None:  # the oracle's own code for these bytes
        L, C = oracle.codebook(oracle.histogram(x))
        assert np.array_equal(np.asarray(enc.codebook.host.lengths), L)
    else:
        L = np.asarray(cb.host.lengths)
        C = oracle.canonical_codes(L)
    s_or, off_or, _ = oracle.encode(x, B, L, C)
    assert np.array_equal(enc.stream.cpu().numpy(), s_or)
    assert np.array_equal(enc.block_off.cpu().numpy().view(np.uint64), off_or)
    y, e = selfsync(hc, enc.stream, x.size, enc, enc.block_off)
    assert e == 0
    assert torch.equal(y, xd)
    return enc


@pytest.mark.parametrize("kind", ["zipf", "uniform", "skewed", "fp32", "const"])
@pytest.mark.parametrize("B", [16, 4096, 65536, 1 * MIB, 4 * MIB])
def test_selfsync_matches_input(hc, oracle, kind, B):
    """Ragged sizes; B = 4 MiB is one block larger than the input (256 pieces)."""
    check(hc, oracle, data(kind, 3 * MIB + 5 * 4, 11), B, tag=kind)


@pytest.mark.parametrize("n", [1, 15, 16, 17, 255, 4097, 65536 + 3])
def test_selfsync_small_and_ragged(hc, oracle, n):
    for B in (16, 4096, 1 * MIB):
        check(hc, oracle, synth.zipf_bytes(n, 1.1, n), B, tag="small")


@pytest.mark.parametrize("m", [14, 33, 65])
def test_selfsync_long_codes(hc, oracle, m):
    """Fibonacci counts: codes of up to m-1 bits (table fallback, 64-bit codes)."""
    fib = [1, 1]
    while len(fib) < m:
        fib.append(fib[-1] + fib[-2])
    h = np.zeros(256, np.uint64)
    h[:m] = fib
    cb = hc.DeviceCodebook(hc.hc_build_codebook(h))
    assert cb.max_len == m - 1
    x = np.random.default_rng(m).integers(0, m, size=600_001).astype(np.uint8)
    for B in (65536, 1 * MIB):
        check(hc, oracle, x, B, cb=cb, tag=f"fib{m}")


def test_selfsync_workload_segment(hc, oracle):
    """64 MiB segments of the benchmark's kinds at its block size: the result
    equals the input (a property that holds at any size)."""
    for t, kind in enumerate(synth.SEGMENT_KINDS):
        xd = synth.segment_bytes_torch(kind, 64 * MIB, synth.derive_seed(3, t))
        enc = hc.compress(xd, 65536)
        y, e = selfsync(hc, enc.stream, xd.numel(), enc, enc.block_off)
        assert e == 0 and torch.equal(y, xd), kind


@pytest.mark.parametrize("kind", ["zipf", "skewed"])
def test_selfsync_rejects_corruption(hc, oracle, kind):
    x = synth.zipf_bytes(200_000, 1.2, 1) if kind == "zipf" else synth.skewed_bytes(200_000, 1)
    B = 4096
    enc = hc.compress(dev(x), B)
    L = np.asarray(enc.codebook.host.lengths)
    s0 = enc.stream.cpu().numpy()
    off = enc.block_off.cpu().numpy().view(np.uint64)
    bits = np.array([int.from_bytes(s0[int(o):int(o) + 4].tobytes(), "little") for o in off[:-1]])
    cases = {}
    s = s0.copy(); s[int(off[5])] ^= 1; cases["header bit"] = s
    s = s0.copy(); s[int(off[-2]) + 3] = 0x7F; cases["header too large"] = s
    i = next(i for i in range(bits.size) if bits[i] % 32)
    pb = int(bits[i]); w = int(off[i]) + 4 + 4 * (pb // 32); pos = 31 - pb % 32
    s = s0.copy(); s[w + pos // 8] |= 1 << (pos % 8); cases["nonzero pad"] = s
    s = s0.copy(); s[int(off[7]) + 4 + 40] ^= 0x10; cases["payload bit"] = s
    cases["truncated"] = s0[:-4].copy()
    cases["trailing"] = np.concatenate([s0, np.zeros(4, np.uint8)])
    for name, s in cases.items():
        st_or = oracle.decode_status(s, x.size, B, L)[0]
        sd = dev(s)
        nb = hc.num_blocks(x.size, B)
        offd = torch.zeros(nb + 1, dtype=torch.int64, device="cuda")
        err = hc.new_error_word("cuda")
        hc.hc_walk_blocks(sd, sd.numel(), nb, offd, err)
        st_gpu = hc.read_error(err)
        y = None
        if st_gpu == 0:
            y, st_gpu = selfsync(hc, sd, x.size, enc, offd)
        if st_or == oracle.ERR_CORRUPT:
            assert st_gpu == hc.HC_ERR_CORRUPT, name
        else:  # a payload flip may still decode; then both give the same bytes
            assert st_or == 0 and st_gpu == 0, name
            assert np.array_equal(y.cpu().numpy(), oracle.decode(s, x.size, B, L)), name
    # wrong symbol count
    n2 = x.size + B
    nb2 = hc.num_blocks(n2, B)
    off2 = torch.zeros(nb2 + 1, dtype=torch.int64, device="cuda")
    off2[: off.size] = enc.block_off
    off2[off.size:] = enc.block_off[-1]
    _, st = selfsync(hc, enc.stream, n2, enc, off2)
    assert st == hc.HC_ERR_CORRUPT


def test_selfsync_argument_errors(hc):
    x = dev(synth.zipf_bytes(1000, 1.2, 3))
    enc = hc.compress(x, 64)
    out = torch.empty(1008, dtype=torch.uint8, device="cuda")
    err = hc.new_error_word("cuda")
    with pytest.raises(hc.HcError):
        hc.hc_decode_blocks_selfsync(enc.stream, enc.nbytes, 1000, 24, enc.codebook, enc.block_off, out, err)
    with pytest.raises(hc.HcError):
        hc.hc_decode_blocks_selfsync(enc.stream, enc.nbytes - 1, 1000, 64, enc.codebook, enc.block_off, out, err)
    with pytest.raises(hc.HcError):
        hc.hc_decode_blocks_selfsync(enc.stream, enc.nbytes, 1000, 64, enc.codebook, enc.block_off, out[1:], err)


def _fib_codebook(hc, m):
    fib = [1, 1]
    while len(fib) < m:
        fib.append(fib[-1] + fib[-2])
    h = np.zeros(256, np.uint64)
    h[:m] = fib
    return hc.DeviceCodebook(hc.hc_build_codebook(h))


def batch_decode(hc, encs, ns, B):
    """hc_decode_batch_selfsync over the encodings; returns outputs and status."""
    items = hc.make_items(len(encs))
    ys = []
    for k, (enc, n) in enumerate(zip(encs, ns)):
        ys.append(torch.empty(max(n, 16), dtype=torch.uint8, device="cuda"))
        hc.set_item(items, k, x=enc.stream, n=n, in_bytes=enc.nbytes, dcb=enc.codebook, out=ys[k],
                    block_off=enc.block_off)
    ws = torch.empty(max(hc.hc_batch_workspace_bytes(items, B), 256), dtype=torch.uint8, device="cuda")
    err = hc.new_error_word("cuda")
    hc.hc_decode_batch_selfsync(items, B, ws, err)
    return [y[:n] for y, n in zip(ys, ns)], hc.read_error(err)


@pytest.mark.parametrize("B", [4096, 65536, 1 * MIB])
def test_selfsync_batch_matches_oracle(hc, oracle, B):
    """One call over streams of every code class (complete 8-bit codes by the
    copy form, codes of <= 8 .. 64 bits by the piece decoder), empty and
    ragged sizes: every stream equals the oracle's encoding of its input and
    every output equals the input."""
    rng = np.random.default_rng(B)
    xs, cbs = [], []
    kinds = ["uniform", "skewed", "fp32", "zipf", "const", "fib14", "fib33", "fib65"]
    for k in range(32):
        kind = kinds[k % len(kinds)]
        n = int(rng.integers(0, 3 * B + 17)) if k % 5 else int(rng.integers(0, 40))
        if kind.startswith("fib"):
            m = int(kind[3:])
            cb = _fib_codebook(hc, m)
            x = rng.integers(0, m, size=n).astype(np.uint8)
        else:
            cb = None
            x = data(kind, (n + 3) // 4 * 4, 100 + k)[:n]
        xs.append(x)
        cbs.append(cb)
    print(f"[selfsync] batch B={B}: {len(xs)} streams, {sum(x.size for x in xs)} bytes", flush=True)
    xd = [dev(x) for x in xs]
    encs = [hc.compress(x, B, codebook=cb) if x.size else hc.compress(x, B, codebook=cb or _fib_codebook(hc, 14))
            for x, cb in zip(xd, cbs)]
    for k, (x, enc) in enumerate(zip(xs, encs)):
        if x.size == 0:
            continue
        L = np.asarray(enc.codebook.host.lengths)
        s_or, off_or, _ = oracle.encode(x, B, L, oracle.canonical_codes(L))
        assert np.array_equal(enc.stream.cpu().numpy(), s_or), k
        assert np.array_equal(enc.block_off.cpu().numpy().view(np.uint64), off_or), k
    ys, e = batch_decode(hc, encs, [x.size for x in xs], B)
    assert e == 0
    for k in range(len(xs)):
        assert torch.equal(ys[k], xd[k]), k


def test_selfsync_batch_workload_segments(hc, oracle):
    """The benchmark's three kinds, 64 MiB each, in one batched call at its
    block size: the outputs equal the inputs."""
    xd = [synth.segment_bytes_torch(kind, 64 * MIB, synth.derive_seed(3, t)) for t, kind in enumerate(synth.SEGMENT_KINDS)]
    encs = [hc.compress(x, 65536) for x in xd]
    ys, e = batch_decode(hc, encs, [x.numel() for x in xd], 65536)
    assert e == 0
    for k in range(len(xd)):
        assert torch.equal(ys[k], xd[k]), k


def test_selfsync_batch_rejects_corruption(hc, oracle):
    """A payload bit flip the oracle rejects, in one stream of a batch: the
    call reports CORRUPT; the other streams still decode to their inputs."""
    B = 4096
    x = synth.skewed_bytes(200_000, 5)
    enc = hc.compress(dev(x), B)
    L = np.asarray(enc.codebook.host.lengths)
    s0 = enc.stream.cpu().numpy()
    off = enc.block_off.cpu().numpy().view(np.uint64)
    bad = None
    for pos in range(int(off[3]) + 4, int(off[4])):
        s = s0.copy()
        s[pos] ^= 0x08
        if oracle.decode_status(s, x.size, B, L)[0] == oracle.ERR_CORRUPT:
            bad = s
            break
    assert bad is not None
    good = [hc.compress(dev(synth.zipf_bytes(100_000 + 16 * k, 1.2, k)), B) for k in range(3)]
    broken = hc.Encoded(dev(bad), enc.block_off, None, x.size, B, 0, enc.codebook)
    encs = good[:2] + [broken] + good[2:]
    ns = [g.n for g in good[:2]] + [x.size] + [g.n for g in good[2:]]
    ys, e = batch_decode(hc, encs, ns, B)
    assert e == hc.HC_ERR_CORRUPT
    for k in (0, 1, 3):
        assert torch.equal(ys[k], hc.decompress(encs[k])), k


def test_decode_without_index_complete8(hc, oracle):
    """hc_decode_blocks without an index on complete 8-bit codes: the copy
    form cuts blocks into chunks itself (no index needed when every code has
    8 bits); ragged blocks, against the oracle's decode, and a header that
    disagrees with 8 bits per symbol is rejected."""
    cb8 = hc.DeviceCodebook(hc.hc_codebook_from_lengths(np.full(256, 8, np.uint8)))
    for n, B in ((1_000_003, 4096), (300_001, 65536), (5000, 16), (777, 144)):
        x = synth.uniform_bytes(n, n)
        xd = dev(x)
        enc = hc.compress(xd, B, codebook=cb8)
        assert enc.codebook.max_len == 8 and enc.codebook.host.nsym == 256
        L = np.asarray(enc.codebook.host.lengths)
        s_or, _, _ = oracle.encode(x, B, L, oracle.canonical_codes(L))
        assert np.array_equal(enc.stream.cpu().numpy(), s_or)
        y = torch.empty(max(n, 16), dtype=torch.uint8, device="cuda")[:n]
        err = hc.new_error_word("cuda")
        hc.hc_decode_blocks(enc.stream, enc.nbytes, n, B, enc.codebook, enc.block_off, None, 0, y, err)
        assert hc.read_error(err) == 0 and torch.equal(y, xd), (n, B)
    s = enc.stream.cpu().numpy().copy()
    s[0] ^= 0x08  # the first header: 8 bits more than the block holds
    assert oracle.decode_status(s, x.size, B, L)[0] == oracle.ERR_CORRUPT
    err = hc.new_error_word("cuda")
    hc.hc_decode_blocks(dev(s), s.size, x.size, B, enc.codebook, enc.block_off, None, 0, y, err)
    assert hc.read_error(err) == hc.HC_ERR_CORRUPT
