"""Checks of the seeded input generators (shapes, closed-form counts, reproducibility)."""
import math

import numpy as np

import synth


def test_splitmix64_reference_values():
    # SplitMix64 with state 0 advanced by the golden gamma: first outputs of the published
    # generator (state += 0x9E3779B97F4A7C15, then the two multiply-xorshift rounds)
    got = synth.bits(0, 3).tolist()
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_uniform_ranges_and_moments():
    u = synth.uniform(5, 200000, -1.0, 1.0)
    assert u.min() >= -1.0 and u.max() < 1.0
    assert abs(u.mean()) < 0.01 and abs((u * u).mean() - 1 / 3) < 0.01
    r = synth.randint(6, 100000, -3, 3)
    assert r.min() == -3 and r.max() == 3
    assert np.array_equal(synth.uniform(5, 10, 0, 1), synth.uniform(5, 10, 0, 1))
    assert np.array_equal(synth.uniform(5, 10, 0, 1, offset=4)[:6], synth.uniform(5, 14, 0, 1)[4:10])


def _sorted_unique_rows(A):
    for i in range(A.nrows):
        c = A.col[A.rowptr[i]:A.rowptr[i + 1]]
        if c.size and not np.all(c[1:] > c[:-1]):
            return False
    return True


def test_laplacian_counts_and_symmetry():
    A = synth.laplacian2d(64)
    assert A.nnz == 64 * 64 + 4 * 64 * 63 == 20224
    B = synth.laplacian3d(9)
    assert B.nnz == 7 * 9 ** 3 - 6 * 9 ** 2
    for M in (A, B):
        D = M.dense()
        assert np.array_equal(D, D.T)
        assert _sorted_unique_rows(M)


def test_anderson_counts_and_disorder():
    L = 16
    A = synth.anderson3d(L)
    assert A.nnz == 7 * L ** 3 and np.all(A.row_lengths() == 7)
    D = A.dense()
    assert np.array_equal(D - np.diag(np.diag(D)), (D - np.diag(np.diag(D))).T)
    d = np.diag(D)
    assert d.min() >= -8.25 and d.max() <= 8.25 and d.std() > 4.0
    off = A.val[A.col != np.repeat(np.arange(A.nrows), 7)]
    assert np.all(off == -1.0)
    assert _sorted_unique_rows(A)


def test_irregular_shape():
    n = 50000
    A = synth.irregular(n, seed=3)
    lens = A.row_lengths()
    assert lens.min() >= 1 and lens.max() <= 2000
    assert abs(lens.mean() - 15.0) < 0.6
    assert _sorted_unique_rows(A)
    assert A.col.min() >= 0 and A.col.max() < n
    # about half of the entries lie in the +-5000 band
    rows = np.repeat(np.arange(n), lens)
    near = np.abs(A.col.astype(np.int64) - rows) <= 5000
    assert 0.5 < near.mean() < 0.65
    assert abs(A.val.mean()) < 0.02 and abs(A.val.std() - 1) < 0.02
    B = synth.irregular(n, seed=3)
    assert np.array_equal(A.col, B.col) and np.array_equal(A.val, B.val)


def test_batch_edges():
    e = synth.laplacian3d_batch()
    assert len(e) == 64 and min(e) >= 20 and max(e) <= 100
    assert sum(x ** 3 for x in e) > 0


def test_normal_moments():
    z = synth.normal(9, 400000)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1) < 0.01
    assert abs(np.mean(np.abs(z) < 1) - math.erf(1 / math.sqrt(2))) < 0.005
