"""GPU parity of the wave-staged decoder (chunks of at most 128 symbols).

The encoder's stream, offsets and index are compared with the oracle byte for
byte, and the decode with the input, for every code shape the staged decoder
has a variant for (codes of <= 8, <= 10, <= 12 bits from the table; 13..16
bits through the canonical ranges; 17..24 bits in rounds of 8 symbols), at
index strides from 16 to 128, with ragged blocks and chunks, with stream and
output not on a 128-byte line, and with corrupt streams and indexes, which
both sides must reject.
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


def roundtrip(hc, oracle, x: np.ndarray, B: int, S: int, tag: str, cb=None):
    print(f"[stage] {tag} n={x.size} B={B} S={S}", flush=True)
    xd = dev(x)
    if cb is None:
        h = oracle.histogram(x)
        L, C = oracle.codebook(h)
        dcb = hc.DeviceCodebook(hc.hc_build_codebook(h))
    else:
        L, C = cb.lengths, cb.codes
        dcb = hc.DeviceCodebook(cb)
    enc = hc.compress(xd, B, sub_block=S, codebook=dcb)
    s_or, off_or, _ = oracle.encode(x, B, L, C)
    assert np.array_equal(u64(enc.block_off), off_or)
    assert np.array_equal(enc.stream.cpu().numpy(), s_or)
    assert np.array_equal(u32(enc.sub_idx)[: hc.hc_sub_index_entries(x.size, B, S)], oracle.sub_index(x, B, S, L))
    y = hc.decompress(enc)
    assert torch.equal(y, xd)
    return enc


@pytest.mark.parametrize("S", [16, 48, 64, 112, 128])
@pytest.mark.parametrize("kind", ["zipf", "skewed", "fp32"])
def test_kinds_and_strides(hc, oracle, kind, S):
    n = 1 * MIB + (4100 if kind == "fp32" else 4099)  # fp32 bytes come in fours
    x = synth.zipf_bytes(n, 1.1, S) if kind == "zipf" else synth.segment_bytes(kind, n, S)
    for B in (4096, 65536, 4096 + 16 * 7):
        roundtrip(hc, oracle, x, B, S, kind)


@pytest.mark.parametrize("n", [1, 15, 16, 17, 127, 128, 129, 8191, 65537])
def test_ragged(hc, oracle, n):
    x = synth.zipf_bytes(n, 1.3, n)
    roundtrip(hc, oracle, x, 4096, 128, "ragged")
    roundtrip(hc, oracle, x, 160, 32, "ragged small blocks")


def test_single_symbol_and_all_equal(hc, oracle):
    roundtrip(hc, oracle, np.full(70_001, 7, np.uint8), 4096, 128, "single symbol")
    x = np.tile(np.arange(256, dtype=np.uint8), 512)
    np.random.default_rng(4).shuffle(x)
    roundtrip(hc, oracle, x, 16384, 128, "all 256 equal (copy launch)")


@pytest.mark.parametrize("m", [11, 13, 16, 17, 20, 25])
def test_code_lengths_per_variant(hc, oracle, m):
    """Fibonacci counts: codes of m-1 bits, frequent in the data, so the
    long-code ranges (13..16) and the 8-symbol rounds (17..24) run, and the
    wave's chunks no longer fit its area at once (several passes)."""
    fib = [1, 1]
    while len(fib) < m:
        fib.append(fib[-1] + fib[-2])
    h = np.zeros(256, np.uint64)
    h[:m] = fib
    cb = hc.hc_build_codebook(h)
    assert cb.max_len == m - 1
    x = np.random.default_rng(m).integers(0, m, size=200_003).astype(np.uint8)
    for B, S in ((4096, 128), (65536, 64), (2048, 16)):
        roundtrip(hc, oracle, x, B, S, f"fib{m}", cb=cb)


@pytest.mark.parametrize("kind", ["zipf", "skewed", "fp32"])
@pytest.mark.parametrize("shift_in,shift_out", [(16, 0), (48, 32), (112, 80)])
def test_unaligned_lines(hc, oracle, kind, shift_in, shift_out):
    n = 300_012 if kind == "fp32" else 300_013
    x = synth.zipf_bytes(n, 1.2, 5) if kind == "zipf" else synth.segment_bytes(kind, n, 5)
    B, S = 16384, 128
    enc = roundtrip(hc, oracle, x, B, S, f"{kind} unaligned {shift_in}/{shift_out}")
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


def _decode(hc, enc, stream_np=None, sub=None):
    err = hc.new_error_word("cuda")
    s = enc.stream if stream_np is None else dev(stream_np)
    out = torch.empty(max(enc.n, 16), dtype=torch.uint8, device="cuda")
    hc.hc_decode_blocks(s, s.numel(), enc.n, enc.block_size, enc.codebook, enc.block_off,
                        enc.sub_idx if sub is None else sub, enc.sub_block, out, err)
    torch.cuda.synchronize()
    return hc.read_error(err), out


@pytest.mark.parametrize("kind", ["zipf", "skewed"])
def test_corruption(hc, oracle, kind):
    x = synth.zipf_bytes(200_000, 1.2, 1) if kind == "zipf" else synth.skewed_bytes(200_000, 1)
    B, S = 4096, 128
    enc = hc.compress(dev(x), B, sub_block=S)
    L = enc.codebook.host.lengths
    s0 = enc.stream.cpu().numpy()
    off = u64(enc.block_off)
    assert _decode(hc, enc)[0] == 0
    bits = np.array([int.from_bytes(s0[int(o):int(o) + 4].tobytes(), "little") for o in off[:-1]])
    cases = {}
    s = s0.copy(); s[int(off[5])] ^= 1; cases["header bit"] = s
    i = next(i for i in range(bits.size) if bits[i] % 32)
    pb = int(bits[i]); w = int(off[i]) + 4 + 4 * (pb // 32); pos = 31 - pb % 32
    s = s0.copy(); s[w + pos // 8] |= 1 << (pos % 8); cases["nonzero pad"] = s
    # payload bit flips inside chunks: the oracle decides whether each one is detectable
    rng = np.random.default_rng(9)
    for k in range(6):
        blk = int(rng.integers(0, bits.size))
        p = int(rng.integers(0, int(bits[blk])))
        s = s0.copy(); s[int(off[blk]) + 4 + 4 * (p // 32) + (31 - p % 32) // 8] ^= 1 << ((31 - p % 32) % 8)
        cases[f"payload flip {k}"] = s
    for name, s in cases.items():
        st_or, y_or = oracle.decode_status(s, x.size, B, L)
        st_gpu, y = _decode(hc, enc, stream_np=s)
        if st_or != 0:
            # the chunks cover the block's bits back to back, so a stream the
            # oracle rejects cannot decode chunk by chunk either
            assert st_gpu == hc.HC_ERR_CORRUPT, name
        else:
            # a flip that still parses: the index may no longer fall on code
            # starts (rejected), else the one parse of a prefix code is the oracle's
            assert st_gpu in (0, hc.HC_ERR_CORRUPT), name
            if st_gpu == 0:
                assert np.array_equal(y[: x.size].cpu().numpy(), y_or), name
    # indexes that disagree with the stream: a shifted entry, one past the block, one before its predecessor
    nidx, cpb = hc.hc_sub_index_entries(x.size, B, S), B // S
    for j, delta in ((1, 1), (3, -1), (40, 5000), (nidx - cpb - 1, 1)):  # the last: a full block's last chunk
        bad = enc.sub_idx.clone()
        bad[j] += delta
        assert _decode(hc, enc, sub=bad)[0] == hc.HC_ERR_CORRUPT, (j, delta)


def test_batch_mixed_kinds(hc, oracle):
    """hc_decode_batch with S = 128 over streams of every kind (the complete
    8-bit codes in the copy launch, the rest in the staged launch)."""
    B, S = 65536, 128
    xs = [synth.segment_bytes(k, 2 * MIB + 16 * i, 30 + i) for i, k in enumerate(["uniform", "skewed", "fp32", "skewed"])]
    xs.append(synth.zipf_bytes(3 * MIB + 48, 1.05, 77))
    encs = [roundtrip(hc, oracle, x, B, S, f"batch item {i}") for i, x in enumerate(xs)]
    items = hc.make_items(len(xs))
    outs = [torch.full((x.size + 64,), 0xEE, dtype=torch.uint8, device="cuda") for x in xs]
    for k, (x, e) in enumerate(zip(xs, encs)):
        hc.set_item(items, k, x=e.stream, n=x.size, in_bytes=e.nbytes, dcb=e.codebook, out=outs[k][: x.size],
                    block_off=e.block_off, sub_idx=e.sub_idx)
    ws = torch.empty(hc.hc_batch_workspace_bytes(items, B), dtype=torch.uint8, device="cuda")
    err = hc.new_error_word("cuda")
    hc.hc_decode_batch(items, B, S, ws, err)
    torch.cuda.synchronize()
    assert hc.read_error(err) == 0
    for x, o in zip(xs, outs):
        oo = o.cpu().numpy()
        assert np.array_equal(oo[: x.size], x) and (oo[x.size:] == 0xEE).all()
