"""The parameters the autotuner chooses change no output byte: the encode
tile (hc_tuning.encode_tile_loads) leaves stream, offsets and index as the
oracle's, and the index stride S (which picks the decoder) leaves the
stream and the decoded bytes unchanged."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1107_1525_amd as hc_mod

    return hc_mod


@pytest.mark.parametrize("B", [16384, 65536, 262144])
@pytest.mark.parametrize("kind", ["zipf", "skewed", "fp32"])
def test_tile_loads_change_no_byte(hc, oracle, B, kind):
    n = 3 * (1 << 20) + 4100
    x = synth.zipf_bytes(n, 1.1, 3) if kind == "zipf" else synth.segment_bytes(kind, n, 3)
    xd = torch.from_numpy(x).cuda()
    L, C = oracle.codebook(oracle.histogram(x))
    s_or, off_or, _ = oracle.encode(x, B, L, C)
    idx_or = oracle.sub_index(x, B, 128, L)
    cb = hc.DeviceCodebook(hc.hc_build_codebook(oracle.histogram(x)))
    try:
        for q in (0, 1, 2, 4):
            hc.hc_set_tuning(q)
            assert hc.hc_get_tuning()["encode_tile_loads"] == q
            enc = hc.compress(xd, B, sub_block=128, codebook=cb)
            assert np.array_equal(enc.block_off.cpu().numpy().view(np.uint64), off_or), q
            assert np.array_equal(enc.stream.cpu().numpy(), s_or), q
            assert np.array_equal(enc.sub_idx.cpu().numpy().view(np.uint32)[: idx_or.size], idx_or), q
            assert torch.equal(hc.decompress(enc), xd), q
    finally:
        hc.hc_set_tuning(0)


def test_index_stride_changes_no_decoded_byte(hc):
    x = torch.from_numpy(synth.segment_bytes("fp32", 2 * (1 << 20), 8)).cuda()
    outs = []
    for S in (0, 64, 128, 1024):
        enc = hc.compress(x, 65536, sub_block=S)
        outs.append((enc.stream.clone(), hc.decompress(enc)))
    for s_, y in outs:
        assert torch.equal(s_, outs[0][0]) and torch.equal(y, x)


def test_tuning_rejects_bad_values(hc):
    with pytest.raises(hc.HcError):
        hc.hc_set_tuning(3)
    assert hc.hc_get_tuning()["encode_tile_loads"] == 0
