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


@pytest.mark.parametrize("b", [1, 2, 4, 8])
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
