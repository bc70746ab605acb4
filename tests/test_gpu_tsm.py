"""GPU parity of the tall-skinny block-vector kernels against the oracle (FP64)."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sc():
    import torch

    import paper_1507_08101_amd as sc

    assert torch.cuda.is_available()
    sc.lib()
    return sc


@pytest.mark.parametrize("n,m,k", [(0, 3, 2), (1, 1, 1), (1000, 8, 8), (100003, 5, 3), (20000, 64, 64),
                                   (7777, 17, 40)])
@pytest.mark.parametrize("kahan", [False, True])
def test_tsmttsm(sc, n, m, k, kahan):
    V = synth.block_vector(n, m, 160)
    W = synth.block_vector(n, k, 161)
    X0 = synth.block_vector(m, k, 162)
    Xd = dev(X0)
    sc.sell_tsmttsm(dev(V), dev(W), Xd, alpha=2.0, beta=-0.5, kahan=kahan)
    ref = oracle.tsmttsm(V, W, 2.0, -0.5, X0, kahan=kahan)
    scale = 2.0 * np.abs(V).T @ np.abs(W) + 0.5 * np.abs(X0)
    assert np.all(np.abs(host(Xd) - ref) <= 1e-12 * scale + 1e-300)


def test_tsmttsm_kahan_accuracy_on_gpu(sc):
    n = 200000
    a = synth.normal(163, n) * np.exp(synth.uniform(164, n, -15, 15))
    V = np.stack([a, np.ones(n)], axis=1)
    W = np.stack([synth.normal(165, n), -np.ones(n) * 1e-3], axis=1)
    Xd = dev(np.zeros((2, 2)))
    sc.sell_tsmttsm(dev(V), dev(W), Xd, kahan=True)
    X = host(Xd)
    for l in range(2):
        for j in range(2):
            exact = math.fsum((V[:, l] * W[:, j]).tolist())
            bound = 4.5e-16 * abs(exact) + 1.2e-16 * float(np.sum(np.abs(V[:, l] * W[:, j])))
            assert abs(X[l, j] - exact) <= bound


@pytest.mark.parametrize("m,k", [(8, 8), (4, 12), (16, 4)])
@pytest.mark.parametrize("kahan", [False, True])
def test_tsmttsm_aligned_path_equals_element_path(sc, m, k, kahan):
    """m and k multiples of 4 with 16-byte aligned rows take the 16-byte-load kernel; the same
    values in a buffer shifted by one double (rows 8 bytes off alignment) take the per-element
    kernel. Both visit every thread's rows in the same order: equal bit for bit, and within the
    oracle's bound."""
    import torch

    n = 123457
    V = synth.block_vector(n, m, 170 + m)
    W = synth.block_vector(n, k, 180 + k)
    out = []
    for off in (0, 1):
        vb = torch.zeros(n * m + 2, dtype=torch.float64, device="cuda:0")
        wb = torch.zeros(n * k + 2, dtype=torch.float64, device="cuda:0")
        Vd = vb[off:off + n * m].view(n, m)
        Wd = wb[off:off + n * k].view(n, k)
        Vd.copy_(dev(V))
        Wd.copy_(dev(W))
        assert (Vd.data_ptr() % 16 == 0) == (off == 0)
        Xd = torch.zeros((m, k), dtype=torch.float64, device="cuda:0")
        sc.sell_tsmttsm(Vd, Wd, Xd, kahan=kahan)
        out.append(host(Xd))
    assert np.array_equal(out[0], out[1])
    ref = oracle.tsmttsm(V, W, 1.0, 0.0, np.zeros((m, k)), kahan=kahan)
    assert np.all(np.abs(out[0] - ref) <= 1e-12 * (np.abs(V).T @ np.abs(W)) + 1e-300)


def test_tsmttsm_deterministic(sc):
    import torch

    V = dev(synth.block_vector(300001, 4, 166))
    W = dev(synth.block_vector(300001, 4, 167))
    X1 = torch.zeros((4, 4), dtype=torch.float64, device="cuda:0")
    X2 = torch.zeros_like(X1)
    sc.sell_tsmttsm(V, W, X1)
    sc.sell_tsmttsm(V, W, X2)
    torch.cuda.synchronize()
    assert torch.equal(X1, X2)


@pytest.mark.parametrize("n,m,k", [(1, 1, 1), (50000, 8, 8), (12345, 3, 17), (4096, 64, 64)])
def test_tsmm(sc, n, m, k):
    V = synth.block_vector(n, m, 168)
    X = synth.block_vector(m, k, 169)
    W0 = synth.block_vector(n, k, 170)
    Wd = dev(W0)
    sc.sell_tsmm(dev(V), dev(X), Wd, alpha=0.5, beta=2.0)
    ref = oracle.tsmm(V, X, 0.5, 2.0, W0)
    scale = 0.5 * np.abs(V) @ np.abs(X) + 2.0 * np.abs(W0)
    assert np.all(np.abs(host(Wd) - ref) <= 1e-13 * scale + 1e-300)


@pytest.mark.parametrize("n,m", [(1, 1), (50001, 8), (9999, 3), (3000, 64)])
def test_tsmm_inplace(sc, n, m):
    V = synth.block_vector(n, m, 171)
    X = synth.block_vector(m, m, 172)
    Vd = dev(V)
    sc.sell_tsmm_inplace(Vd, dev(X), alpha=1.5, beta=-0.5)
    ref = oracle.tsmm_inplace(V, X, 1.5, -0.5)
    scale = 1.5 * np.abs(V) @ np.abs(X) + 0.5 * np.abs(V)
    assert np.all(np.abs(host(Vd) - ref) <= 1e-13 * scale + 1e-300)
