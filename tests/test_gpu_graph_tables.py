"""Captured batch calls against code tables that change between replays.

The batch calls shape their launches (kernel variant, tile and table sizes)
from every item's code when called; a HIP graph replays those launches as
captured.  A replay whose tables keep their shape decodes and encodes as the
eager calls do; one whose longest code grew, or whose complete 8-bit code
stopped being complete, must report HC_ERR_TABLE_CHANGED instead of running
kernels sized for other tables."""
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


def _setup(hc, B, S):
    xs = [synth.zipf_bytes(300_000, 1.2, 11), synth.segment_bytes("uniform", 200_000, 12),
          synth.segment_bytes("skewed", 250_000, 13)]
    xd = [torch.from_numpy(x).cuda() for x in xs]
    dcbs = [hc.DeviceCodebook(hc.hc_build_codebook(np.bincount(x, minlength=256).astype(np.uint64))) for x in xs]
    outs = [torch.zeros(hc.hc_encode_bound(x.size, B, d.max_len) + 16, dtype=torch.uint8, device="cuda")
            for x, d in zip(xs, dcbs)]
    offs = [torch.zeros(hc.num_blocks(x.size, B) + 1, dtype=torch.int64, device="cuda") for x in xs]
    subs = [torch.zeros(hc.hc_sub_index_entries(x.size, B, S), dtype=torch.int32, device="cuda") for x in xs]
    ys = [torch.zeros(x.size, dtype=torch.uint8, device="cuda") for x in xs]
    e_items, d_items = hc.make_items(3), hc.make_items(3)
    for k in range(3):
        hc.set_item(e_items, k, x=xd[k], dcb=dcbs[k], out=outs[k], block_off=offs[k], sub_idx=subs[k])
    ws = torch.empty(hc.hc_batch_workspace_bytes(e_items, B), dtype=torch.uint8, device="cuda")
    err = hc.new_error_word("cuda")
    hc.hc_encode_batch(e_items, B, S, ws, err)
    C = [int(o[-1].item()) for o in offs]
    for k in range(3):
        hc.set_item(d_items, k, x=outs[k], n=xs[k].size, in_bytes=C[k], dcb=dcbs[k], out=ys[k], block_off=offs[k],
                    sub_idx=subs[k])
    hc.hc_decode_batch(d_items, B, S, ws, err)
    torch.cuda.synchronize()
    assert hc.read_error(err) == 0
    assert all(torch.equal(y, x) for y, x in zip(ys, xd))
    # the items hold raw pointers: every buffer they name lives as long as they do
    return xs, xd, dcbs, outs, ys, e_items, d_items, ws, err, (offs, subs)


@pytest.mark.parametrize("change", ["longer", "not_complete8"])
def test_replay_with_changed_tables(hc, change):
    B, S = 16384, 128
    xs, xd, dcbs, outs, ys, e_items, d_items, ws, err, keep = _setup(hc, B, S)
    g, gd = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()  # encode + decode, and decode alone
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=side):
        hc.hc_encode_batch(e_items, B, S, ws, err)
        hc.hc_decode_batch(d_items, B, S, ws, err)
    torch.cuda.synchronize()
    with torch.cuda.graph(gd, stream=side):
        hc.hc_decode_batch(d_items, B, S, ws, err)
    torch.cuda.synchronize()
    for y in ys:
        y.zero_()
    g.replay()
    torch.cuda.synchronize()
    assert hc.read_error(err) == 0
    assert all(torch.equal(y, x) for y, x in zip(ys, xd))  # same tables: the replay is the eager result
    if change == "longer":
        # buffer 0's code gets longer than the launches were shaped for
        L = np.zeros(256, np.uint8)
        L[:21] = list(range(1, 21)) + [20]
        k, cb = 0, hc.hc_codebook_from_lengths(L)
        assert cb.max_len > max(d.max_len for d in dcbs)
    else:
        # buffer 1's complete 8-bit code (its own decode launch) becomes an
        # incomplete code of the same longest length
        L = np.zeros(256, np.uint8)
        L[0] = 1
        L[1:129] = 8
        k, cb = 1, hc.hc_codebook_from_lengths(L)
        assert cb.max_len == 8 and cb.nsym < 256
    dcbs[k].update(cb)
    torch.cuda.synchronize()
    err.zero_()
    # the longer code is met first by the encode's length pass; the incomplete
    # code by the decode's copy launch, and by the encode's launches for
    # complete 8-bit codes (which run no length pass)
    (g if change == "longer" else gd).replay()
    torch.cuda.synchronize()
    assert hc.read_error(err) == hc.HC_ERR_TABLE_CHANGED
    if change == "not_complete8":
        err.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert hc.read_error(err) == hc.HC_ERR_TABLE_CHANGED
