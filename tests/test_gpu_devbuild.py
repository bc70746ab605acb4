"""GPU tests of the construction on the device: for every matrix, chunk height and sorting
window, the device-built SELL-C-sigma arrays (permutation, chunk lengths and starts, columns,
values in the storage type) equal the host builder's bit for bit, the host builder's layout
itself being pinned to the oracle's brute-force layout; invalid input is rejected."""
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

    assert torch.cuda.is_available()
    sc.lib()
    return sc


def _mats():
    return {
        "empty": synth.CSR(0, 0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0), "empty"),
        "one": synth.CSR(1, 1, np.array([0, 1], np.int64), np.zeros(1, np.int32), np.array([2.5]), "one"),
        "lap2d_64": synth.laplacian2d(64),
        "anderson_12": synth.anderson3d(12),
        "irregular_20000": synth.irregular(20000, band=1000, max_len=700, seed=71),
        "random_ragged": synth.random_sparse(333, 257, 0.03, 72, empty_rows=17, long_row=257, duplicates=True),
        "zero_rows": synth.CSR(50, 10, np.zeros(51, np.int64), np.zeros(0, np.int32), np.zeros(0), "zero_rows"),
    }


MATS = _mats()


def _dev_csr(A):
    import torch

    return (torch.from_numpy(np.ascontiguousarray(A.rowptr, dtype=np.int64)).cuda(),
            torch.from_numpy(np.ascontiguousarray(A.col, dtype=np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(A.val, dtype=np.float64)).cuda())


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("C,sigma", [(1, 1), (8, 1), (32, 1), (32, 32), (32, 1024), (64, 10 ** 9), (12, 7)])
@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
def test_device_build_equals_host_build(sc, name, C, sigma, dt):
    A = MATS[name]
    Mh = sc.SellMatrix.from_csr(A, C=C, sigma=sigma, dtype=dt)
    rp, co, va = _dev_csr(A)
    Md = sc.SellMatrix.from_device_csr(A.nrows, A.ncols, rp, co, va, C=C, sigma=sigma, dtype=dt)
    ih, idv = dict(Mh.info), dict(Md.info)
    assert ih == idv, (ih, idv)
    eh, ed = Mh.export_sell(), Md.export_sell()  # (perm, cl, cs, col, val)
    for k in range(5):
        assert np.array_equal(eh[k], ed[k]), k
    # and the layout is the oracle's
    perm, cl, cs = oracle.sell_layout(A, C, min(sigma, max(A.nrows, 1)))
    assert np.array_equal(ed[0], perm) and np.array_equal(ed[1], cl) and np.array_equal(ed[2], cs)
    # the CSR comes back bit for bit (values in the storage type)
    rp2, col2, val2 = Md.export_csr()
    assert np.array_equal(rp2, A.rowptr) and np.array_equal(col2, A.col)
    Mh.close()
    Md.close()


@pytest.mark.parametrize("b", [1, 8])
def test_device_built_matrix_products(sc, b):
    import torch

    A = MATS["irregular_20000"]
    rp, co, va = _dev_csr(A)
    M = sc.SellMatrix.from_device_csr(A.nrows, A.ncols, rp, co, va, C=32, sigma=256)
    X = synth.block_vector(A.ncols, b, 73)
    Y = torch.zeros((A.nrows, b), dtype=torch.float64, device="cuda:0")
    sc.sell_spmmv(M, dev(X), Y)
    assert colwise_relerr(host(Y), oracle.spmmv(A, X), abs_product(A, X)) <= 1e-12
    # values-only update and the transposed product work on a device-built matrix
    newv = synth.uniform(74, A.nnz, -1, 1)
    M.update_values(dev(newv))
    A2 = synth.CSR(A.nrows, A.ncols, A.rowptr, A.col, newv)
    sc.sell_spmmv(M, dev(X), Y)
    assert colwise_relerr(host(Y), oracle.spmmv(A2, X), abs_product(A2, X)) <= 1e-12
    XT = synth.block_vector(A.nrows, b, 75)
    YT = torch.zeros((A.ncols, b), dtype=torch.float64, device="cuda:0")
    sc.sell_spmmv_T(M, dev(XT), YT, deterministic=True)
    assert colwise_relerr(host(YT), oracle.spmmv_T(A2, XT)) <= 1e-12
    M.close()


def test_device_build_rejects_invalid_csr(sc):
    A = MATS["random_ragged"]
    rp, co, va = _dev_csr(A)
    bad = co.clone()
    bad[5] = A.ncols  # column out of range
    with pytest.raises(sc.SellError):
        sc.SellMatrix.from_device_csr(A.nrows, A.ncols, rp, bad, va)
    bad = co.clone()
    bad[-1] = -3
    with pytest.raises(sc.SellError):
        sc.SellMatrix.from_device_csr(A.nrows, A.ncols, rp, bad, va)
    rpb = rp.clone()
    rpb[10] = rpb[12] + 1  # decreasing row pointers
    with pytest.raises(sc.SellError):
        sc.SellMatrix.from_device_csr(A.nrows, A.ncols, rpb, co, va)
    rpb = rp.clone()
    rpb[0] = 1
    with pytest.raises(sc.SellError):
        sc.SellMatrix.from_device_csr(A.nrows, A.ncols, rpb, co, va)
    # the library is still usable afterwards
    M = sc.SellMatrix.from_device_csr(A.nrows, A.ncols, rp, co, va)
    M.close()


def test_device_build_full_size_anderson128(sc):
    """The benchmark's matrix (2,097,152 rows), with a sorting window: equal to the host build."""
    A = synth.anderson3d(128)
    rp, co, va = _dev_csr(A)
    for sigma in (1, 4096):
        Mh = sc.SellMatrix.from_csr(A, C=32, sigma=sigma)
        Md = sc.SellMatrix.from_device_csr(A.nrows, A.ncols, rp, co, va, C=32, sigma=sigma)
        eh, ed = Mh.export_sell(), Md.export_sell()
        for k in range(5):
            assert np.array_equal(eh[k], ed[k]), (sigma, k)
        Mh.close()
        Md.close()
