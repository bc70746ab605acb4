"""GPU tests of gathering x through the LDS page cache (sell_set_stage): the staged product
sums the same entries of a row in the same order with the same x values, so y and z must equal
the unstaged product's bit for bit, for every fixed width, value type, tile order and a mix of
staged and unstaged tiles. The dots group the rows differently when a workgroup takes its
tiles one at a time, so they agree within the dot bound (1e-12 of sum |u_i v_i|); the FP64
result also matches the oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import abs_product, colwise_relerr, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sc():
    import torch

    import paper_1507_08101_amd as sc

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    sc.lib()
    return sc


def _mats():
    return {
        "anderson_24": (synth.anderson3d(24), 32, 1),           # periodic: wrap-around pages
        "lap3d_30": (synth.laplacian3d(30), 32, 1),
        "lap2d_100": (synth.laplacian2d(100), 32, 1),
        "irregular_20000": (synth.irregular(20000, band=300, max_len=300, seed=31), 32, 64),  # many unstaged tiles
        "ragged_3001": (synth.random_sparse(3001, 3001, 0.002, 32, empty_rows=40, long_row=200), 32, 128),
        "rect_4000x2500": (synth.random_sparse(4000, 2500, 0.0015, 33, empty_rows=9), 16, 1),
    }


MATS = _mats()


def _run(sc, M, X, Y0, Z0, flags, vt):
    import torch

    b = X.shape[1]
    Y, Z = Y0.clone(), Z0.clone()
    dot = torch.full((3 * b,), -3.0, dtype=torch.float64, device="cuda:0")
    if flags is None:
        sc.sell_spmmv(M, X, Y)
    else:
        sc.sell_spmmv_aug(M, X, Y, Z, flags=flags, dot=dot, alpha=0.5, beta=-1.0, gamma=0.25, delta=2.0, eta=-0.5)
    return host(Y), host(Z), host(dot)


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
def test_staged_equals_unstaged(sc, name, dt):
    import torch

    A, C, sigma = MATS[name]
    vt = torch.float64 if dt == "f64" else torch.float32
    M = sc.SellMatrix.from_csr(A, C=C, sigma=sigma, dtype=dt)
    square = A.nrows == A.ncols
    for b in (1, 2, 4, 8, 16, 32):
        X = dev(synth.block_vector(A.ncols, b, 600 + b), vt)
        Y0 = dev(synth.block_vector(A.nrows, b, 700 + b), vt)
        Z0 = dev(synth.block_vector(A.nrows, b, 800 + b), vt)
        for flags in (None, sc.SCALE | sc.AXPBY | sc.DOT_YY | sc.CHAIN | (sc.SHIFT | sc.DOT_XY | sc.DOT_XX if square else 0)):
            M.set_stage(0, 0)
            ref = _run(sc, M, X, Y0, Z0, flags, vt)
            for stage, stride in ((1, 0), (1, 2), (1, 3), (0, 2)):
                M.set_stage(stage, stride)
                got = _run(sc, M, X, Y0, Z0, flags, vt)
                assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), (name, dt, b, flags, stage, stride)
                if flags is not None:
                    y, x = ref[0], host(X)[:A.nrows] if square else None
                    sums = [np.sum(np.abs(y * y), axis=0)]
                    if square:
                        sums += [np.sum(np.abs(x * y), axis=0), np.sum(x * x, axis=0)]
                    for g, sm in enumerate(sums):
                        seg = slice(g * b, (g + 1) * b)
                        assert np.all(np.abs(got[2][seg] - ref[2][seg]) <= 1e-12 * sm), (name, dt, b, stage, stride, g)
            if dt == "f64" and flags is None:
                Xh = host(X)
                assert colwise_relerr(got[0], oracle.spmmv(A, Xh), abs_product(A, Xh)) <= 1e-12
    M.close()


def test_staged_kpm_full_size(sc):
    """The benchmark's recurrence (128^3 Anderson, SELL-32-1, b = 8) with x through LDS, with and
    without the stride that makes a workgroup sweep the planes of its tile column: the last
    vectors equal the unstaged run's bit for bit (every step's y does), the moments agree within
    the dot bound of their inner products."""
    import torch

    A = synth.anderson3d(128)
    s = (6 + 16.5 / 2) / 0.99
    b, Mst = 8, 6
    V0 = synth.block_vector(A.nrows, b, synth.SEED_X)
    M = sc.SellMatrix.from_csr(A, C=32, sigma=1)
    out = []
    for stage, stride in ((0, 0), (1, 0), (1, 64), (0, 64)):
        M.set_stage(stage, stride)
        V = dev(V0)
        W = torch.zeros_like(V)
        mu = torch.zeros((2 * Mst + 1) * b, dtype=torch.float64, device="cuda:0")
        last = sc.sell_kpm(M, V, W, Mst, s, 0.0, mu)
        out.append((host(mu), host(W if last else V)))
    for got in out[1:]:
        assert np.array_equal(got[1], out[0][1])
        # each moment is 2 <v_p, v_q> - mu_0 or mu_1 with |<v_p, v_q>| <= ||v_0||^2
        nx2 = np.sum(V0 * V0, axis=0)
        assert np.all(np.abs(got[0] - out[0][0]).reshape(-1, b) <= 3e-12 * nx2)
    M.close()


def test_stage_setter_rejects(sc):
    A = synth.laplacian2d(10)
    M = sc.SellMatrix.from_csr(A)
    for bad in ((2, 0), (-1, 0), (1, -3)):
        with pytest.raises(sc.SellError):
            M.set_stage(*bad)
    M.close()
