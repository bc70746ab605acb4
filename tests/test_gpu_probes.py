"""GPU tests of the measurement probes: the streaming bandwidth probes and the random-gather
probe run on valid buffers and reject invalid arguments before any launch."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sc():
    import torch

    import paper_1507_08101_amd as sc

    assert torch.cuda.is_available()
    sc.lib()
    return sc


def test_bandwidth_probes_run(sc):
    import torch

    a = torch.ones(1 << 20, dtype=torch.float32, device="cuda")
    b = torch.zeros_like(a)
    sc.sell_probe_bandwidth(0, b, a, a.numel() * 4)
    torch.cuda.synchronize()
    assert torch.equal(a, b)  # the nontemporal copy copies
    sc.sell_probe_bandwidth(3, b, a * 2, a.numel() * 4)
    torch.cuda.synchronize()
    assert torch.equal(b, a * 2)
    for kind in (1, 2, 4):
        sc.sell_probe_bandwidth(kind, b, a, a.numel() * 4)
    torch.cuda.synchronize()
    with pytest.raises(sc.SellError):
        sc.sell_probe_bandwidth(5, b, a, 1024)
    with pytest.raises(sc.SellError):
        sc.sell_probe_bandwidth(0, b, a, 1000)  # not a multiple of 16


@pytest.mark.parametrize("reads,writes", [(0, 1), (1, 0), (1, 1), (2, 1), (3, 1), (4, 0), (4, 1)])
@pytest.mark.parametrize("unroll,nt", [(1, 0), (4, 1), (8, 0)])
def test_stream_probe_sums_its_reads(sc, reads, writes, unroll, nt):
    import torch

    n4 = 100_003  # float4 elements per stream: a ragged tail for every grid below
    src = torch.arange(4 * n4 * 4, dtype=torch.float32, device="cuda").remainder_(97.0) if reads else None
    for grid in (1, 7, 1000):
        dst = torch.zeros(max(n4, grid) * 4, dtype=torch.float32, device="cuda")
        sc.sell_probe_stream(reads, writes, unroll, nt, grid, dst, src, n4 * 16)
        torch.cuda.synchronize()
        if reads:
            s = src[: reads * n4 * 4].view(reads, n4, 4).sum(dim=0)
        else:
            s = torch.tensor([1.0, 2.0, 3.0, 4.0], device="cuda").expand(n4, 4)
        if writes:
            assert torch.equal(dst[: n4 * 4].view(n4, 4), s), grid
        else:
            got = dst[: grid * 4].view(grid, 4).double().sum(dim=0)
            assert torch.allclose(got, s.double().sum(dim=0), rtol=1e-5), grid


def test_stream_probe_rejects(sc):
    import torch

    a = torch.zeros(4096, dtype=torch.float32, device="cuda")
    for args in ((0, 0, 1, 0, 8), (5, 1, 1, 0, 8), (1, 2, 1, 0, 8), (1, 1, 3, 0, 8), (1, 1, 1, 0, 0)):
        with pytest.raises(sc.SellError):
            sc.sell_probe_stream(*args, a, a, 1024)
    with pytest.raises(sc.SellError):
        sc.sell_probe_stream(1, 1, 1, 0, 8, a, a, 1000)  # not a multiple of 16
    with pytest.raises(sc.SellError):
        sc.sell_probe_stream(1, 1, 1, 0, 8, a, None, 1024)  # reads without a source


@pytest.mark.parametrize("b", [1, 2, 4, 8, 16, 32])
def test_gather_probe_runs(sc, b):
    import torch

    n = 100_003
    x = torch.rand((n, b), dtype=torch.float64, device="cuda")
    idx = torch.randint(-5, n + 5, (1_000_001,), dtype=torch.int32, device="cuda")  # out of range reads row 0
    sink = torch.zeros(1, dtype=torch.float64, device="cuda")
    sc.sell_probe_gather(x, idx, sink)
    sc.sell_probe_gather(x, idx[:7], sink)  # only the tail loop
    sc.sell_probe_gather(x, idx[:0], sink)  # nothing to do
    torch.cuda.synchronize()
    assert sink.item() == 0.0


def test_gather_probe_rejects(sc):
    import torch

    x = torch.rand((1000, 3), dtype=torch.float64, device="cuda")  # 24-byte rows
    idx = torch.zeros(10, dtype=torch.int32, device="cuda")
    sink = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(sc.SellError):
        sc.sell_probe_gather(x, idx, sink)
    with pytest.raises(sc.SellError):
        sc.sell_probe_gather(x[:, :1].contiguous(), idx.long(), sink)  # int64 indices
