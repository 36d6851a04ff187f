"""Host-resident pipeline (transfers overlapped with the coding, one code per
chunk) against the CPU oracle: every chunk's stream, offsets and sub-block
index bit-exact, chunks back to back in the host buffer, and the round trip
through the pipeline's decompress."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

KIB = synth.KIB


@pytest.fixture(scope="module")
def hc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1107_1525_amd as hc_mod

    return hc_mod


def pinned(x: np.ndarray) -> torch.Tensor:
    t = torch.empty(max(x.size, 16), dtype=torch.uint8).pin_memory()[: x.size]
    t.copy_(torch.from_numpy(np.ascontiguousarray(x)))
    return t


def mixed_host(nchunks: int, M: int, tail: int, seed: int) -> np.ndarray:
    parts = [synth.segment_bytes(synth.mixed_kind(t), M, synth.derive_seed(seed, t)) for t in range(nchunks)]
    if tail:
        parts.append(synth.zipf_bytes(tail, 1.2, synth.derive_seed(seed, nchunks)))
    return np.concatenate(parts) if parts else np.zeros(0, np.uint8)


@pytest.mark.parametrize("B,S,M,slots,nchunks,tail", [
    (4096, 1024, 256 * KIB, 3, 5, 100 * KIB + 7),   # more chunks than slots, ragged last chunk and block
    (4096, 0, 64 * KIB, 2, 4, 0),                   # two slots, no sub-block index
    (16384, 4096, 1024 * KIB, 3, 1, 0),             # a single chunk
    (4096, 1024, 256 * KIB, 3, 0, 1000),            # one short chunk
])
def test_host_pipeline_matches_oracle(hc, oracle, B, S, M, slots, nchunks, tail):
    from paper_1107_1525_amd.hostpipe import HostPipeline, plan_chunks

    x = mixed_host(nchunks, M, tail, 77 + nchunks)
    xh = pinned(x)
    pipe = HostPipeline(B, S, chunk_bytes=M, slots=slots)
    enc = pipe.compress(xh)
    plan = plan_chunks(x.size, M, B)
    assert [(c.start, c.n) for c in enc.chunks] == plan
    data = enc.data.numpy()
    pos = 0
    for c in enc.chunks:
        xs = x[c.start:c.start + c.n]
        L, Cw = oracle.codebook(oracle.histogram(xs))
        s_o, off_o, _ = oracle.encode(xs, B, L, Cw)
        assert np.array_equal(c.lengths, L), c.start
        pos = (pos + 15) // 16 * 16  # each chunk from a 16-byte boundary, in order
        assert c.pos == pos and c.nbytes == s_o.size, c.start
        assert np.array_equal(data[c.pos:c.pos + c.nbytes], s_o), c.start
        assert np.array_equal(c.block_off.numpy().view(np.uint64), off_o), c.start
        if S:
            assert np.array_equal(c.sub_idx.numpy().view(np.uint32), oracle.sub_index(xs, B, S, L)), c.start
        pos += c.nbytes
    assert enc.total == pos
    y = pipe.decompress(enc)
    assert np.array_equal(y.numpy(), x)
    # a second pass through the same pipeline (slots reused) gives the same result
    enc2 = pipe.compress(xh)
    assert enc2.total == enc.total
    d2 = enc2.data.numpy()
    for c, c2 in zip(enc.chunks, enc2.chunks):
        assert (c2.pos, c2.nbytes) == (c.pos, c.nbytes)
        assert np.array_equal(d2[c2.pos:c2.pos + c2.nbytes], data[c.pos:c.pos + c.nbytes])
    assert np.array_equal(pipe.decompress(enc2).numpy(), x)


def test_host_pipeline_empty_input(hc):
    from paper_1107_1525_amd.hostpipe import HostPipeline

    pipe = HostPipeline(4096, 1024, chunk_bytes=64 * KIB)
    enc = pipe.compress(torch.empty(0, dtype=torch.uint8).pin_memory())
    assert enc.total == 0 and enc.chunks == []
    assert pipe.decompress(enc).numel() == 0


def test_host_pipeline_output_too_small(hc):
    from paper_1107_1525_amd.hostpipe import HostPipeline

    x = mixed_host(3, 64 * KIB, 0, 91)  # uniform chunk first: about 64 KiB of stream
    pipe = HostPipeline(4096, 0, chunk_bytes=64 * KIB)
    small = torch.empty(32 * KIB, dtype=torch.uint8).pin_memory()
    with pytest.raises(hc.HcError) as e:
        pipe.compress(pinned(x), out=small)
    assert e.value.status == hc.HC_ERR_NO_SPACE
    # the pipeline stays usable after the refusal
    enc = pipe.compress(pinned(x))
    assert np.array_equal(pipe.decompress(enc).numpy(), x)
