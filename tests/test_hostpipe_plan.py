"""Chunk plan of the host-resident pipeline (no GPU): whole chunks of M
bytes and one short last chunk, covering the buffer once; M a positive
multiple of the block size, so chunk boundaries are block boundaries."""
import pytest


def plan_chunks():
    from paper_1107_1525_amd.hostpipe import plan_chunks as f

    return f


@pytest.mark.parametrize("n,M,B", [(0, 64, 16), (1, 64, 16), (64, 64, 16), (65, 64, 16), (1000, 128, 32),
                                   (4 << 30, 64 << 20, 65536)])
def test_chunks_cover_the_buffer(n, M, B):
    plan = plan_chunks()(n, M, B)
    assert sum(m for _, m in plan) == n
    pos = 0
    for k, (a, m) in enumerate(plan):
        assert a == pos and 0 < m <= M
        assert a % B == 0  # a chunk's blocks are the buffer's blocks
        if k + 1 < len(plan):
            assert m == M
        pos += m
    assert len(plan) == (n + M - 1) // M


@pytest.mark.parametrize("M,B", [(0, 16), (48, 32), (64, 0), (-64, 16)])
def test_bad_chunk_sizes(M, B):
    with pytest.raises(ValueError):
        plan_chunks()(100, M, B)
