"""Roofline probes through the C ABI: the copy reproduces its source byte for
byte and the read folds exactly the source's 32-bit words (xor, checked on
the host), at sizes below one wave, with a ragged grid-stride tail, and over
many work-groups.  Also the streaming copy hc_copy between device memory and
pinned host memory, and its refusals."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1107_1525_amd as hc_mod

    return hc_mod


@pytest.mark.parametrize("n", [0, 16, 4096 + 48, (1 << 20) + 16 * 37, 64 << 20])
def test_probe_copy_and_read(hc, n):
    g = torch.Generator(device="cuda")
    g.manual_seed(1107 + n)
    x = torch.randint(0, 256, (max(n, 16),), dtype=torch.uint8, device="cuda", generator=g)[:n]
    y = torch.full((max(n, 16),), 0xA5, dtype=torch.uint8, device="cuda")[:n]
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    hc.hc_probe_copy(x, y)
    hc.hc_probe_read(x, sink)
    torch.cuda.synchronize()
    assert torch.equal(x, y)
    want = np.bitwise_xor.reduce(x.cpu().numpy().view(np.uint32)) if n else np.uint32(0)
    assert int(sink.cpu().numpy().view(np.uint32)[0]) == int(want)


def test_probe_rejects_bad_arguments(hc):
    x = torch.zeros(64, dtype=torch.uint8, device="cuda")
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(hc.HcError):
        hc.hc_probe_copy(x[:40], torch.empty(40, dtype=torch.uint8, device="cuda"))  # not a multiple of 16
    with pytest.raises(hc.HcError):
        hc.hc_probe_copy(x[:48], x[16:])  # overlapping
    with pytest.raises(hc.HcError):
        hc.hc_probe_read(x[4:36], sink)  # misaligned


@pytest.mark.parametrize("n", [16, 4096 + 48, (1 << 20) + 16 * 37, 64 << 20])
def test_copy_device_and_pinned_host(hc, n):
    g = torch.Generator(device="cuda")
    g.manual_seed(n)
    d = torch.randint(0, 256, (n + 64,), dtype=torch.uint8, device="cuda", generator=g)
    h = torch.zeros(n + 64, dtype=torch.uint8).pin_memory()
    # device -> pinned host, from an offset inside both allocations
    hc.hc_copy(d[16:16 + n], h[32:32 + n])
    torch.cuda.synchronize()
    assert torch.equal(h[32:32 + n], d[16:16 + n].cpu())
    assert int(h[:32].sum()) == 0 and int(h[32 + n:].sum()) == 0  # nothing outside the range
    # pinned host -> device, and device -> device
    d2 = torch.zeros(n, dtype=torch.uint8, device="cuda")
    hc.hc_copy(h[32:32 + n], d2)
    d3 = torch.zeros(n, dtype=torch.uint8, device="cuda")
    hc.hc_copy(d2, d3)
    torch.cuda.synchronize()
    assert torch.equal(d2, d[16:16 + n]) and torch.equal(d3, d2)


def test_copy_refusals(hc):
    d = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    pageable = torch.zeros(4096, dtype=torch.uint8)  # not pinned: the device cannot reach it
    with pytest.raises(hc.HcError):
        hc.hc_copy(d, pageable)
    with pytest.raises(hc.HcError):
        hc.hc_copy(pageable, d)
    with pytest.raises(hc.HcError):
        hc.hc_copy(d[4:36], torch.zeros(32, dtype=torch.uint8, device="cuda"))  # misaligned
    with pytest.raises(hc.HcError):
        hc.hc_copy(d[:64], d[32:96])  # overlapping


def test_copy_refuses_range_past_its_allocation(hc):
    """A range that starts in an allocation and runs past its end is refused
    on the host (nothing is launched), device or pinned host memory alike."""
    import ctypes

    d = torch.zeros(64 << 20, dtype=torch.uint8, device="cuda")
    d2 = torch.zeros(64 << 20, dtype=torch.uint8, device="cuda")
    h = torch.zeros(1 << 20, dtype=torch.uint8).pin_memory()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    big = 1 << 30  # far past any of these allocations
    for src, dst in ((d, d2), (h, d2), (d, h)):
        rc = hc._lib.hc_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), big, stream)
        assert rc == hc.HC_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert int(d2.count_nonzero()) == 0
    # the same buffers within their sizes copy
    d[:4096] = 7
    hc.hc_copy(d[:4096], h[:4096])
    torch.cuda.synchronize()
    assert bool((h[:4096] == 7).all())
