"""GPU tests of sell_spmmv_aug_noalloc, the augmented product for callers that cannot allocate:
it must give sell_spmmv_aug's results bit for bit (same kernels, same launch), on two calls in a
row where the second has a smaller input, without any allocation by the library, also on a
stream that has never run a product (where sell_spmmv_aug would allocate its workspace), and
under HIP graph capture."""
import numpy as np
import pytest

import synth
from gpu_util import dev, host

pytestmark = pytest.mark.gpu

SCALARS = dict(alpha=0.5, beta=-1.0, gamma=0.25, delta=2.0, eta=-0.5)


@pytest.fixture(scope="module")
def sc():
    import torch

    import paper_1507_08101_amd as sc

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    sc.lib()
    return sc


def _operands(A, b, seed):
    X = dev(synth.block_vector(A.ncols, b, seed))
    Y = dev(synth.block_vector(A.nrows, b, seed + 1))
    Z = dev(synth.block_vector(A.nrows, b, seed + 2))
    return X, Y, Z


def _run(sc, fn, M, X, Y0, Z0, flags):
    import torch

    b = X.shape[1]
    Y, Z = Y0.clone(), Z0.clone()
    dot = torch.full((3 * b,), -3.0, dtype=torch.float64, device="cuda:0")
    fn(M, X, Y, Z, flags=flags, dot=dot, **SCALARS)
    return host(Y), host(Z), host(dot)


def _same(a, b):
    return all(np.array_equal(p, q) for p, q in zip(a, b))


CASES = [  # (matrix, C, sigma, b): a large case, then a smaller one on the next call
    (lambda: synth.irregular(60000, band=2000, max_len=400, seed=41), 32, 1024, 8),
    (lambda: synth.anderson3d(12), 32, 1, 3),
]


@pytest.mark.parametrize("flags", [0, 0xFF & ~0x02, 0x10 | 0x20 | 0x40 | 0x04 | 0x08])
def test_noalloc_matches_aug_two_calls(sc, flags):
    import torch

    for make, C, sigma, b in CASES:
        A = make()
        M = sc.SellMatrix.from_csr(A, C=C, sigma=sigma)
        X, Y0, Z0 = _operands(A, b, 500)
        ref = _run(sc, sc.sell_spmmv_aug, M, X, Y0, Z0, flags)
        live = sc.sell_debug_live_allocs()
        side = torch.cuda.Stream()  # a stream that has never run a product
        with torch.cuda.stream(side):
            sc.sell_debug_fail_alloc(1)  # any allocation by the library now fails
            try:
                got = _run(sc, sc.sell_spmmv_aug_noalloc, M, X, Y0, Z0, flags)
            finally:
                sc.sell_debug_fail_alloc(0)
        assert sc.sell_debug_live_allocs() == live
        assert _same(got, ref), (A.name, b, flags)
        M.close()


def test_noalloc_wide_and_sliced_blocks(sc):
    # b = 70 runs as several launches of at most 64 columns, one after the other on the stream;
    # a slice width of 16 splits b = 32 into two launches
    A = synth.random_sparse(3001, 3001, 0.003, 71, empty_rows=40, long_row=700)
    M = sc.SellMatrix.from_csr(A, C=32, sigma=128)
    flags = 0xFF & ~0x02
    for b, sl in ((70, 0), (32, 16), (1, 0)):
        M.set_slice(sl)
        X, Y0, Z0 = _operands(A, b, 510)
        ref = _run(sc, sc.sell_spmmv_aug, M, X, Y0, Z0, flags)
        got = _run(sc, sc.sell_spmmv_aug_noalloc, M, X, Y0, Z0, flags)
        assert _same(got, ref), (b, sl)
    M.close()


def test_noalloc_low_precision_values(sc):
    import torch

    A = synth.laplacian3d(20)
    for dt in ("f32", "bf16"):
        M = sc.SellMatrix.from_csr(A, C=32, sigma=1, dtype=dt)
        X, Y0, Z0 = (t.to(torch.float32) for t in _operands(A, 8, 520))
        flags = 0xFF & ~0x02
        ref = _run(sc, sc.sell_spmmv_aug, M, X, Y0, Z0, flags)
        got = _run(sc, sc.sell_spmmv_aug_noalloc, M, X, Y0, Z0, flags)
        assert _same(got, ref), dt
        M.close()


def test_noalloc_under_graph_capture(sc):
    """The use it is for: captured into a HIP graph on torch's capture stream and replayed, with
    eager work and synchronisation between the replays; every replay against the eager result."""
    import torch

    A = synth.anderson3d(16)
    M = sc.SellMatrix.from_csr(A, C=32, sigma=1)
    b = 4
    X, Y0, Z0 = _operands(A, b, 530)
    flags = sc.SCALE | sc.SHIFT | sc.AXPBY | sc.DOTS | sc.CHAIN
    ref = _run(sc, sc.sell_spmmv_aug, M, X, Y0, Z0, flags)
    Y, Z = Y0.clone(), Z0.clone()
    dot = torch.zeros(3 * b, dtype=torch.float64, device="cuda:0")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sc.sell_spmmv_aug_noalloc(M, X, Y, Z, flags=flags, dot=dot, **SCALARS)
    for rep in range(3):
        Y.copy_(Y0)
        Z.copy_(Z0)
        dot.fill_(-3.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = (host(Y), host(Z), host(dot))
        assert _same(got, ref), rep
        # eager work on the same array between replays
        _run(sc, sc.sell_spmmv_aug_noalloc, M, X, Y0, Z0, flags)
    del g
    M.close()


def test_noalloc_argument_errors(sc):
    import torch

    A = synth.laplacian2d(16)
    M = sc.SellMatrix.from_csr(A, C=32, sigma=1)
    X, Y, Z = _operands(A, 2, 540)
    with pytest.raises(sc.SellError):
        sc.sell_spmmv_aug_noalloc(M, X, Y, flags=sc.DOT_YY)  # dots without a dot array
    with pytest.raises(sc.SellError):
        sc.sell_spmmv_aug_noalloc(M, X, X, flags=0)  # y aliases x
    with pytest.raises(sc.SellError):
        sc.sell_spmmv_aug_noalloc(M, X, Y.to(torch.float32), flags=0)  # wrong vector type
    M.close()
