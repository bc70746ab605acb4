"""GPU tests of the parameter choice: the autotuner returns a valid configuration that is at
least as fast as the default one it timed, answers a matrix of the same shape class from its
cache, and the launch parameters it may choose leave every row's result unchanged."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import (abs_product, assert_lowprec_product, colwise_relerr, dev, gamma_bound, host,
                      rounded_matrix, to_oracle_flags)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sc():
    import torch

    import paper_1507_08101_amd as sc

    assert torch.cuda.is_available()
    sc.lib()
    return sc


def test_autotune_choice_and_cache(sc):
    A = synth.laplacian3d(40)
    t = sc.sell_autotune(A, 8, "f64", cache=False)
    assert t["C"] in (16, 32, 64) and t["sigma"] >= 1 and t["vpt"] in (0, 1, 2, 4)
    assert 0 <= t["blocks_per_cu"] <= 2 and t["trials"] > 5
    assert 0 < t["us"] <= t["default_us"]
    # same family and order of magnitude: answered from the cache
    t2 = sc.sell_autotune(synth.laplacian3d(38), 8, "f64")
    assert t2["trials"] == 0 and (t2["C"], t2["sigma"], t2["vpt"]) == (t["C"], t["sigma"], t["vpt"])
    # another block width is another class
    t3 = sc.sell_autotune(A, 1, "f64")
    assert t3["trials"] > 0


def test_tuned_matrix_parity(sc):
    import torch

    A = synth.irregular(20000, band=2000, max_len=500, seed=61)
    M = sc.SellMatrix.from_csr_tuned(A, 4, "f64")
    X = synth.block_vector(A.ncols, 4, 62)
    Y = torch.zeros((A.nrows, 4), dtype=torch.float64, device="cuda:0")
    sc.sell_spmmv(M, dev(X), Y)
    assert colwise_relerr(host(Y), oracle.spmmv(A, X), abs_product(A, X)) <= 1e-12
    M.close()


@pytest.mark.parametrize("b", [1, 2, 8, 32])
def test_launch_parameters_do_not_change_rows(sc, b):
    import torch

    A = synth.random_sparse(3000, 3000, 0.004, 63, empty_rows=30, long_row=2000)
    M = sc.SellMatrix.from_csr(A, C=32, sigma=128)
    X = dev(synth.block_vector(A.ncols, b, 64))
    ref = None
    for vpt in (0, 1, 2, 4):
        if vpt > b:
            continue
        for bpc, waves in ((0, 0), (1, 0), (2, 0), (5, 0), (0, 2), (0, 8), (1, 16)):
            M.set_launch(vpt, bpc)
            M.set_waves(waves)
            Y = torch.zeros((A.nrows, b), dtype=torch.float64, device="cuda:0")
            dot = torch.zeros(3 * b, dtype=torch.float64, device="cuda:0")
            sc.sell_spmmv_aug(M, X, Y, flags=sc.SHIFT | sc.DOTS, gamma=0.25, dot=dot)
            got = host(Y)
            if ref is None:
                ref = got
                Xh = host(X)
                dref = oracle.spmmv_aug(A, Xh, flags=oracle.SHIFT | oracle.DOT_YY | oracle.DOT_XY | oracle.DOT_XX,
                                        gamma=0.25)[2]
            assert np.array_equal(got, ref), (vpt, bpc, waves)
            den = np.concatenate([np.sum(got * got, 0), np.sum(np.abs(Xh * got), 0), np.sum(Xh * Xh, 0)])
            assert np.all(np.abs(host(dot) - dref) <= 1e-12 * den), (vpt, bpc, waves)
    with pytest.raises(sc.SellError):
        M.set_waves(3)
    with pytest.raises(sc.SellError):
        M.set_launch(3, 0)
    with pytest.raises(sc.SellError):
        M.set_launch(0, 65)
    M.close()


@pytest.mark.parametrize("b,slices", [(32, (0, 8, 16)), (24, (0, 8, 16))])
def test_slices_do_not_change_rows(sc, b, slices):
    """A block processed in column slices (the autotuner's b packing) gives every row bit for bit,
    with per-column shifts, chain and dots landing in their columns."""
    import torch

    A = synth.random_sparse(3000, 3000, 0.004, 65, empty_rows=30, long_row=2000)
    M = sc.SellMatrix.from_csr(A, C=32, sigma=128)
    Xh = synth.block_vector(A.ncols, b, 66)
    Y0 = synth.block_vector(A.nrows, b, 67)
    Z0 = synth.block_vector(A.nrows, b, 68)
    gv = np.linspace(-0.5, 0.5, b)
    fl = sc.VSHIFT | sc.SCALE | sc.AXPBY | sc.DOTS | sc.CHAIN
    kw = dict(alpha=0.75, beta=-0.5, delta=0.25, eta=1.5)
    ref = None
    for sl in slices:
        M.set_slice(sl)
        Y, Z = dev(Y0), dev(Z0)
        dot = torch.zeros(3 * b, dtype=torch.float64, device="cuda:0")
        sc.sell_spmmv_aug(M, dev(Xh), Y, Z, flags=fl, gamma_v=gv, dot=dot, **kw)
        got = (host(Y), host(Z), host(dot))
        if ref is None:
            ref = got
            Yr, Zr, dr = oracle.spmmv_aug(A, Xh, Y0, Z0, flags=oracle.VSHIFT | oracle.SCALE | oracle.AXPBY
                                          | oracle.DOT_YY | oracle.DOT_XY | oracle.DOT_XX | oracle.CHAIN,
                                          gamma_v=gv, **kw)
            scale = 0.75 * (abs_product(A, Xh) + 0.5 * np.abs(Xh)) + 0.5 * np.abs(Y0)
            assert colwise_relerr(got[0], Yr, scale) <= 1e-12
            assert colwise_relerr(got[1], Zr, 0.25 * np.abs(Z0) + 1.5 * np.abs(Yr) + 1.5 * scale) <= 1e-12
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), sl
        Yq = got[0]
        den = np.concatenate([np.sum(Yq * Yq, 0), np.sum(np.abs(Xh * Yq), 0), np.sum(Xh * Xh, 0)])
        assert np.all(np.abs(got[2] - dr) <= 1e-12 * den), sl
    with pytest.raises(sc.SellError):
        M.set_slice(3)
    with pytest.raises(sc.SellError):
        M.set_slice(64)
    M.close()


def test_autotune_reports_slice(sc):
    A = synth.irregular(30000, band=3000, max_len=400, seed=69)
    t = sc.sell_autotune(A, 32, "f64", cache=False)
    assert t["slice"] in (0, 8, 16) and t["waves"] in (0, 1, 2, 4, 8) and t["us"] <= t["default_us"]
    assert t["batch"] in (0, 5, 7, 8)
    M = sc.SellMatrix.from_csr_tuned(A, 32, "f64", cache=True)
    assert M.tune["slice"] == t["slice"] and M.tune["waves"] == t["waves"] and M.tune["batch"] == t["batch"]
    if t["batch"]:
        assert M.info["batch"] == t["batch"]
    import torch

    X = synth.block_vector(A.ncols, 32, 70)
    Y = torch.zeros((A.nrows, 32), dtype=torch.float64, device="cuda:0")
    sc.sell_spmmv(M, dev(X), Y)
    assert colwise_relerr(host(Y), oracle.spmmv(A, X), abs_product(A, X)) <= 1e-12
    M.close()


def _batch_cases():
    return [
        ("random_ragged", lambda: synth.random_sparse(3001, 3001, 0.003, 71, empty_rows=40, long_row=700), 32, 128),
        ("anderson3d_16", lambda: synth.anderson3d(16), 32, 1),
        ("laplacian2d_45", lambda: synth.laplacian2d(45), 32, 1),
    ]


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("case", range(3))
def test_batch_lengths_bit_identical(sc, dt, case):
    """Index batches of 5, 7 and 8 entries give every output bit for bit (each row is summed
    in stored order either way) for the fixed widths and columns per lane, and the FP64 result
    matches the oracle; the augmented product with dots and the chain as well."""
    import torch

    name, make, C, sigma = _batch_cases()[case]
    A = make()
    M = sc.SellMatrix.from_csr(A, C=C, sigma=sigma, dtype=dt)
    vt = torch.float64 if dt == "f64" else torch.float32
    for b, vpts in ((1, (1,)), (2, (1, 2)), (4, (4,)), (8, (1, 2, 4)), (16, (4,)), (32, (4,))):
        X = dev(synth.block_vector(A.ncols, b, 72), vt)
        for vpt in vpts:
            M.set_launch(vpt, 0)
            ref = None
            for bl in (8, 7, 5, 0):
                M.set_batch(bl)
                Y = torch.zeros((A.nrows, b), dtype=vt, device="cuda:0")
                sc.sell_spmmv(M, X, Y)
                got = host(Y)
                if ref is None:
                    ref = got
                    Xh = host(X)
                    if dt == "f64":
                        assert colwise_relerr(got, oracle.spmmv(A, Xh), abs_product(A, Xh)) <= 1e-12, (name, b)
                    else:
                        assert_lowprec_product(got, A, Xh, dt, what=(name, dt, b, vpt))
                assert np.array_equal(got, ref), (name, dt, b, vpt, bl)
    M.set_launch(0, 0)
    b = 8
    X = dev(synth.block_vector(A.ncols, b, 73), vt)
    Y0 = dev(synth.block_vector(A.nrows, b, 74), vt)
    Z0 = dev(synth.block_vector(A.nrows, b, 75), vt)
    fl = sc.SCALE | sc.AXPBY | sc.DOT_YY | sc.DOT_XY | sc.CHAIN | (sc.SHIFT | sc.DOT_XX if A.nrows == A.ncols else 0)
    ref = None
    for bl in (8, 7, 5):
        M.set_batch(bl)
        Y, Z = Y0.clone(), Z0.clone()
        dot = torch.zeros(3 * b, dtype=torch.float64, device="cuda:0")
        sc.sell_spmmv_aug(M, X, Y, Z, flags=fl, alpha=0.5, beta=-1.0, gamma=0.25, delta=0.5, eta=2.0, dot=dot)
        got = (host(Y), host(Z), host(dot))
        if ref is None:
            ref = got
            _check_aug_against_oracle(A, dt, fl, host(X), host(Y0), host(Z0), got)
        assert all(np.array_equal(g, r) for g, r in zip(got, ref)), (name, dt, bl)
    M.close()


def _check_aug_against_oracle(A, dt, fl, X, Y0, Z0, got):
    """The augmented product of the test above (alpha 0.5, beta -1, gamma 0.25, delta 0.5, eta 2)
    against the oracle: FP64 within the normwise 1e-12; FP32/BF16 values with FP32 vectors
    against the exact augmented product of the rounded inputs, per element, within
    gamma_{k+4}(2^-24) (|alpha|(|A~||x| + |gamma||x|) + |beta||y0|) for y (k products, shift,
    scale and axpby, the alpha of the shift counted once more) and |eta| times that plus
    gamma_2 (|delta||z0| + |eta||y|) for the chain; the dots are FP64 sums of the stored y."""
    kw = dict(alpha=0.5, beta=-1.0, gamma=0.25, delta=0.5, eta=2.0)
    oflags = to_oracle_flags(fl)
    Ar = rounded_matrix(A, dt)
    ry, rz, rd = oracle.spmmv_aug(Ar, X, Y=Y0, Z=Z0, flags=oflags, **kw)
    gy, gz, gd = got
    shift = 0.25 if oflags & oracle.SHIFT else 0.0
    scale = 0.5 * (abs_product(Ar, X) + shift * np.abs(X)) + np.abs(Y0)
    if dt == "f64":
        assert colwise_relerr(gy, ry, scale) <= 1e-12
        assert colwise_relerr(gz, rz, 0.5 * np.abs(Z0) + 2.0 * np.abs(ry) + 2.0 * scale) <= 1e-12
    else:
        k = A.row_lengths().reshape(-1, 1)
        by = gamma_bound(k + 4, 2.0 ** -24) * scale
        assert np.all(np.abs(gy - ry) <= by), float(np.max(np.abs(gy - ry) / by))
        bz = 2.0 * by + gamma_bound(2, 2.0 ** -24) * (0.5 * np.abs(Z0) + 2.0 * np.abs(gy))
        assert np.all(np.abs(gz - rz) <= bz), float(np.max(np.abs(gz - rz) / bz))
    b = X.shape[1]
    pairs = [(gy, gy), (X[:A.nrows], gy), (X[:A.nrows], X[:A.nrows])]
    for g, bit in enumerate((oracle.DOT_YY, oracle.DOT_XY, oracle.DOT_XX)):
        if not oflags & bit:
            continue
        u, v = pairs[g]
        ref = np.array([oracle.dot(u[:, j], v[:, j]) for j in range(b)])
        assert np.all(np.abs(gd[g * b:(g + 1) * b] - ref) <= 1e-12 * np.sum(np.abs(u * v), axis=0)), g
