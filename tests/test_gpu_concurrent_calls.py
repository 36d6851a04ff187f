"""Batch calls from several host threads at once, each on its own stream.

A batch call with more than one code class forks its launches onto the
library's side streams and joins them back with events; the fork state is
shared by every call on a device.  Two threads here encode and decode
batches that mix every class (so every call forks) on their own streams,
many times over, and every output is compared with the input and with the
stream the same call makes alone (0 bytes tolerance)."""
import threading

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


def _batch(hc, seed, B, S):
    kinds = ["uniform", "skewed", "fp32", "uniform", "skewed"]
    xs = [synth.segment_bytes(k, 300_000 + 16 * i, seed * 10 + i) for i, k in enumerate(kinds)]
    xd = [torch.from_numpy(x).cuda() for x in xs]
    dcbs = [hc.DeviceCodebook(hc.hc_build_codebook(np.bincount(x, minlength=256).astype(np.uint64))) for x in xs]
    outs = [torch.zeros(hc.hc_encode_bound(x.size, B, d.max_len) + 16, dtype=torch.uint8, device="cuda")
            for x, d in zip(xs, dcbs)]
    offs = [torch.zeros(hc.num_blocks(x.size, B) + 1, dtype=torch.int64, device="cuda") for x in xs]
    subs = [torch.zeros(hc.hc_sub_index_entries(x.size, B, S), dtype=torch.int32, device="cuda") for x in xs]
    ys = [torch.zeros(x.size, dtype=torch.uint8, device="cuda") for x in xs]
    e_items, d_items = hc.make_items(len(xs)), hc.make_items(len(xs))
    for k in range(len(xs)):
        hc.set_item(e_items, k, x=xd[k], dcb=dcbs[k], out=outs[k], block_off=offs[k], sub_idx=subs[k])
    ws = torch.empty(hc.hc_batch_workspace_bytes(e_items, B), dtype=torch.uint8, device="cuda")
    err = hc.new_error_word("cuda")
    hc.hc_encode_batch(e_items, B, S, ws, err)
    torch.cuda.synchronize()
    C = [int(o[-1].item()) for o in offs]
    for k in range(len(xs)):
        hc.set_item(d_items, k, x=outs[k], n=xs[k].size, in_bytes=C[k], dcb=dcbs[k], out=ys[k], block_off=offs[k],
                    sub_idx=subs[k])
    ref = [o[:c].clone() for o, c in zip(outs, C)]
    # every buffer an item points to stays referenced for the batch's lifetime
    return dict(xd=xd, dcbs=dcbs, outs=outs, offs=offs, subs=subs, ys=ys, e_items=e_items, d_items=d_items, ws=ws,
                err=err, C=C, ref=ref)


def test_two_threads_fork_at_once(hc):
    B, S = 16384, 128
    batches = [_batch(hc, s, B, S) for s in (1, 2)]
    failures = []

    def work(bt, rounds=25):
        st = torch.cuda.Stream()
        try:
            with torch.cuda.stream(st):
                for r in range(rounds):
                    for y in bt["ys"]:
                        y.zero_()
                    hc.hc_encode_batch(bt["e_items"], B, S, bt["ws"], bt["err"])
                    hc.hc_decode_batch(bt["d_items"], B, S, bt["ws"], bt["err"])
                    st.synchronize()
                    if hc.read_error(bt["err"]):
                        failures.append(("error", r, hc.read_error(bt["err"])))
                        return
                    for k, (y, x) in enumerate(zip(bt["ys"], bt["xd"])):
                        if not torch.equal(y, x):
                            failures.append(("decode", r, k))
                        if not torch.equal(bt["outs"][k][: bt["C"][k]], bt["ref"][k]):
                            failures.append(("stream", r, k))
        except Exception as e:  # reported to the main thread
            failures.append(("exception", repr(e)))

    threads = [threading.Thread(target=work, args=(bt,)) for bt in batches]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not failures, failures[:10]
