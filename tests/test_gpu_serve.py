"""Serving loop on the GPU: continuous batching with overlapping batches, and
every result identical to the same request served alone (0 bytes tolerance)."""
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


def _data(rng, k):
    n = int(np.exp(rng.uniform(np.log(4096), np.log(4 << 20))))
    kind = synth.mixed_kind(k)
    x = synth.segment_bytes(kind, (n + 3) // 4 * 4, 1000 + k)[:n]
    t = torch.empty(max(n, 16), dtype=torch.uint8, device="cuda")[:n]
    t.copy_(torch.from_numpy(x))
    return t


def test_results_same_alone_and_in_the_mix(hc, oracle):
    from paper_1107_1525_amd.serve import Request, Server

    B, S = 65536, 128
    rng = np.random.default_rng(7)
    alone = {}
    srv = Server(block_size=B, sub_block=S, hbm_budget=512 << 20)
    reqs = []
    t0 = srv.clock()
    arrival = 0.0
    for k in range(48):
        x = _data(rng, k)
        arrival += float(rng.exponential(0.0005))
        if k % 2 == 0:
            r = Request("compress", data=x, arrival=t0 + arrival)
            alone[k] = hc.compress(x, B, sub_block=S)
        else:
            enc = hc.compress(x, B, sub_block=S)
            r = Request("decompress", encoded=enc, arrival=t0 + arrival)
            alone[k] = x
        reqs.append(srv.submit(r))
    done = srv.run_until_idle()
    assert len(done) == len(reqs) and srv.in_use == 0
    assert srv.max_inflight_requests > 1  # batches overlapped on the device
    for k, r in enumerate(reqs):
        assert r.completed >= r.admitted >= r.arrival
        if r.kind == "compress":
            assert torch.equal(r.result.stream, alone[k].stream), k
            assert torch.equal(r.result.block_off, alone[k].block_off), k
            assert torch.equal(r.result.sub_idx, alone[k].sub_idx), k
            assert torch.equal(hc.decompress(r.result), r.data), k
            # the whole stream, offsets and index against the oracle's encoding
            # of the request's data with the oracle's own code for it
            x = r.data.cpu().numpy()
            L, Cw = oracle.codebook(oracle.histogram(x))
            assert np.array_equal(r.result.codebook.host.lengths, L), k
            s_or, off_or, _ = oracle.encode(x, B, L, Cw)
            assert np.array_equal(r.result.stream.cpu().numpy(), s_or), k
            assert np.array_equal(r.result.block_off.cpu().numpy().view(np.uint64), off_or), k
            assert np.array_equal(r.result.sub_idx.cpu().numpy().view(np.uint32)[: hc.hc_sub_index_entries(x.size, B, S)],
                                  oracle.sub_index(x, B, S, L)), k
        else:
            assert torch.equal(r.result, alone[k]), k


def test_budget_limits_concurrency(hc):
    from paper_1107_1525_amd.serve import Request, Server, worst_footprint

    B, S = 65536, 128
    rng = np.random.default_rng(8)
    xs = [_data(rng, k) for k in range(12)]
    fps = [worst_footprint(Request("compress", data=x), B, S) for x in xs]
    srv = Server(block_size=B, sub_block=S, hbm_budget=max(fps) + 1, tables=4)
    for x in xs:
        srv.submit(Request("compress", data=x, arrival=0.0))
    peak = 0
    while not srv.idle:
        srv.step()
        peak = max(peak, srv.in_use)
        assert srv.in_use <= srv.adm.budget
    assert len(srv.done) == 12 and peak <= srv.adm.budget
    assert srv.table_growths == 8  # four resident tables, twelve results held
