"""GPU parity on the full-size synthetic workloads: the 64 x 64 Laplacian with the scalars of
its workload definition, and the 4M-row irregular matrix (lognormal row lengths) at several
sorting windows, value types and block widths, checked row by row on samples and through
properties that hold at any size (dots against exactly rounded sums of the GPU's output)."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import abs_product, assert_lowprec_product, colwise_relerr, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sc():
    import torch

    import paper_1507_08101_amd as sc

    assert torch.cuda.is_available()
    sc.lib()
    return sc


@pytest.mark.parametrize("C", [32, 64])
def test_laplacian64_workload(sc, C):
    """n = 4096, 20,224 nonzeros (4 / -1), x ~ U[-1,1]; y = A x, then
    y = 0.5 (A - 0.1 I) x + 1 * y with fused <x,y> and <y,y>."""
    import torch

    A = synth.laplacian2d(64)
    assert A.nnz == 20224
    x = synth.block_vector(A.nrows, 1, synth.SEED_X)
    y0 = synth.block_vector(A.nrows, 1, synth.SEED_Y)
    M = sc.SellMatrix.from_csr(A, C=C, sigma=1)
    xd, yd = dev(x), torch.zeros((A.nrows, 1), dtype=torch.float64, device="cuda:0")
    sc.sell_spmmv(M, xd, yd)
    assert colwise_relerr(host(yd), oracle.spmmv(A, x), abs_product(A, x)) <= 1e-12
    yd = dev(y0)
    dot = torch.zeros(3, dtype=torch.float64, device="cuda:0")
    sc.sell_spmmv_aug(M, xd, yd, flags=sc.SCALE | sc.SHIFT | sc.AXPBY | sc.DOT_XY | sc.DOT_YY, alpha=0.5,
                      gamma=0.1, beta=1.0, dot=dot)
    ref, _, rd = oracle.spmmv_aug(A, x, Y=y0, flags=oracle.SCALE | oracle.SHIFT | oracle.AXPBY | oracle.DOT_XY
                                  | oracle.DOT_YY, alpha=0.5, gamma=0.1, beta=1.0)
    scale = 0.5 * (abs_product(A, x) + 0.1 * np.abs(x)) + np.abs(y0)
    assert colwise_relerr(host(yd), ref, scale) <= 1e-12
    d = host(dot)
    assert abs(d[0] - rd[0]) <= 1e-12 * rd[0]
    assert abs(d[1] - rd[1]) <= 1e-12 * float(np.sum(np.abs(x * ref)))
    M.close()


_IRR = {}


def _irregular():
    if "A" not in _IRR:
        _IRR["A"] = synth.irregular(4_000_000)
    return _IRR["A"]


def _check_sampled(A, X, Y, rows, vals, tol):
    for i in rows:
        p0, p1 = A.rowptr[i], A.rowptr[i + 1]
        cols = A.col[p0:p1]
        ref = vals[p0:p1] @ X[cols]
        scale = np.abs(vals[p0:p1]) @ np.abs(X[cols])
        assert np.all(np.abs(Y[i] - ref) <= tol * (scale + 1e-300)), i


@pytest.mark.parametrize("sigma,b,dt", [(1, 1, "f64"), (32, 8, "f64"), (1024, 8, "f64"), (10 ** 9, 32, "f64"),
                                        (1024, 8, "bf16"), (10 ** 9, 4, "f32")])
def test_irregular_4M_sampled_rows(sc, sigma, b, dt):
    import torch

    A = _irregular()
    lens = A.row_lengths()
    M = sc.SellMatrix.from_csr(A, C=32, sigma=sigma, dtype=dt)
    info = M.info
    assert info["nnz"] == A.nnz and info["stored"] >= A.nnz
    vt = torch.float64 if dt == "f64" else torch.float32
    X = synth.block_vector(A.ncols, b, synth.SEED_X)
    if dt != "f64":
        X = X.astype(np.float32).astype(np.float64)
    Yd = torch.zeros((A.nrows, b), dtype=vt, device="cuda:0")
    dot = torch.zeros(3 * b, dtype=torch.float64, device="cuda:0")
    sc.sell_spmmv_aug(M, dev(X, vt), Yd, flags=sc.DOT_YY, dot=dot)
    Y = host(Yd)
    rows = np.unique(np.concatenate([synth.randint(78, 3000, 0, A.nrows - 1), [0, A.nrows - 1],
                                     np.argsort(-lens)[:20]]))  # includes the longest rows
    if dt == "f64":
        _check_sampled(A, X, Y, rows, A.val, 1e-12)
    else:
        vals = oracle.round_f32(A.val) if dt == "f32" else oracle.round_bf16(A.val)
        # FP32 accumulation: |err| <= gamma_k |A||x| with k = row length + 1
        k = int(lens[rows].max()) + 1
        u = 2.0 ** -24
        _check_sampled(A, X, Y, rows, vals, k * u / (1 - k * u))
    d = host(dot)
    for j in range(min(b, 4)):
        ref = math.fsum((Y[:, j] * Y[:, j]).tolist())
        assert abs(d[j] - ref) <= 1e-12 * ref
    M.close()


def test_irregular_4M_whole_output_sigma1024_b8(sc):
    """The irregular workload at full size in its fastest configuration (FP64, SELL-32-1024,
    b = 8, the default 16-wave grid): every row of y against the oracle's CSR product, normwise
    per column, and <y, y> within the dot bound."""
    import torch

    A = _irregular()
    b = 8
    M = sc.SellMatrix.from_csr(A, C=32, sigma=1024)
    X = synth.block_vector(A.ncols, b, synth.SEED_X)
    Yd = torch.zeros((A.nrows, b), dtype=torch.float64, device="cuda:0")
    dot = torch.zeros(3 * b, dtype=torch.float64, device="cuda:0")
    sc.sell_spmmv_aug(M, dev(X), Yd, flags=sc.DOT_YY, dot=dot)
    Y = host(Yd)
    M.close()
    R = oracle.spmmv(A, X)
    assert colwise_relerr(Y, R) <= 1e-12
    d = host(dot)[:b]
    ref = np.sum(R * R, axis=0)
    assert np.all(np.abs(d - ref) <= 1e-12 * ref)


def test_irregular_4M_whole_output_bf16_sigma1024_b8(sc):
    """The same at BF16 values with FP32 vectors: every element within the deterministic bound
    of a k-term FP32 sum, gamma_k |A~||x|, against the exact product of the rounded inputs."""
    import torch

    A = _irregular()
    b = 8
    M = sc.SellMatrix.from_csr(A, C=32, sigma=1024, dtype="bf16")
    X32 = synth.block_vector(A.ncols, b, synth.SEED_X).astype(np.float32).astype(np.float64)
    Yd = torch.zeros((A.nrows, b), dtype=torch.float32, device="cuda:0")
    sc.sell_spmmv(M, dev(X32, torch.float32), Yd)
    M.close()
    assert_lowprec_product(host(Yd), A, X32, "bf16", what="irregular 4M bf16 b=8")


def test_batch_64_laplacians_full(sc):
    """The batched workload at full size: 64 3D Dirichlet Laplacians with edges ~ U{20..100}
    (22.2 M rows), 8 right-hand sides each. The batched product (one launch) is checked row by
    row on samples of every matrix; mixed-precision batched CG (BF16 values, FP32 iterations,
    FP64 refinement, HIP graph) must bring every system to ||b - A x|| <= 1e-10 ||b||, with the
    residual recomputed by the oracle from the returned solutions."""
    import torch

    b = 8
    edges = synth.laplacian3d_batch(64)
    mats = [synth.laplacian3d(e) for e in edges]
    M64 = [sc.SellMatrix.from_csr(A, C=32, sigma=1) for A in mats]
    Mbf = [sc.SellMatrix.from_csr(A, C=32, sigma=1, dtype="bf16") for A in mats]
    B64, Bbf = sc.SellBatch(M64), sc.SellBatch(Mbf)
    offs = np.cumsum([0] + [A.nrows for A in mats])
    X = synth.block_vector(int(offs[-1]), b, synth.SEED_X)
    Y = torch.zeros((int(offs[-1]), b), dtype=torch.float64, device="cuda:0")
    sc.sell_batch_spmmv_aug(B64, dev(X), Y)
    Yh = host(Y)
    for k, A in enumerate(mats):
        Xk, Yk = X[offs[k]:offs[k + 1]], Yh[offs[k]:offs[k + 1]]
        rows = np.unique(np.concatenate([synth.randint(80 + k, 40, 0, A.nrows - 1), [0, A.nrows - 1]]))
        _check_sampled(A, Xk, Yk, rows, A.val, 1e-12)
    del Y
    Bs = np.concatenate([synth.block_vector(A.nrows, b, synth.SEED_Y + 1000 * k) for k, A in enumerate(mats)])
    Xd = torch.zeros((int(offs[-1]), b), dtype=torch.float64, device="cuda:0")
    st = sc.sell_batch_cg(B64, Bbf, dev(Bs), Xd, tol=1e-10, maxit=20000, graph=True)
    Xs = host(Xd)
    for k, A in enumerate(mats):
        assert st[k]["converged"] == 1, (k, st[k])
        Bk = Bs[offs[k]:offs[k + 1]]
        R = Bk - oracle.spmmv(A, Xs[offs[k]:offs[k + 1]])
        rel = np.linalg.norm(R, axis=0) / np.linalg.norm(Bk, axis=0)
        assert np.all(rel <= 1.001e-10), (k, rel.max())
    for obj in [B64, Bbf] + M64 + Mbf:
        obj.close()


@pytest.mark.parametrize("waves,slice_width", [(8, 0), (0, 16)])
def test_irregular_4M_autotuned_configuration(sc, waves, slice_width):
    """The irregular matrix in the configurations the autotuner chooses for b = 32 in FP64
    (C = 16, sigma = 4096, a grid of 8 waves; and the block in two 16-column slices), checked on
    sampled rows with the fused <y, y> of every column against a compensated sum of y."""
    import torch

    A = _irregular()
    lens = A.row_lengths()
    b = 32
    M = sc.SellMatrix.from_csr(A, C=16, sigma=4096)
    M.set_waves(waves)
    M.set_slice(slice_width)
    X = synth.block_vector(A.ncols, b, synth.SEED_X)
    Yd = torch.zeros((A.nrows, b), dtype=torch.float64, device="cuda:0")
    dot = torch.zeros(3 * b, dtype=torch.float64, device="cuda:0")
    sc.sell_spmmv_aug(M, dev(X), Yd, flags=sc.DOT_YY, dot=dot)
    Y = host(Yd)
    rows = np.unique(np.concatenate([synth.randint(79, 2000, 0, A.nrows - 1), [0, A.nrows - 1],
                                     np.argsort(-lens)[:20]]))
    _check_sampled(A, X, Y, rows, A.val, 1e-12)
    d = host(dot)
    for j in (0, 15, 16, 31):  # both slices
        ref = math.fsum((Y[:, j] * Y[:, j]).tolist())
        assert abs(d[j] - ref) <= 1e-12 * ref
    M.close()


def test_batch_64_laplacians_mixed_widths_full(sc):
    """The 64 Laplacians with block widths 1, 2, 4, 8, 16, 32 in turn, packed operands, one
    launch (the benchmark's mixed-width row), checked on sampled rows of every matrix."""
    import torch

    edges = synth.laplacian3d_batch(64)
    mats = [synth.laplacian3d(e) for e in edges]
    widths = [(1, 2, 4, 8, 16, 32)[k % 6] for k in range(64)]
    Ms = [sc.SellMatrix.from_csr(A, C=32, sigma=1) for A in mats]
    Bt = sc.SellBatch(Ms)
    Bt.set_widths(widths)
    nx, ny, nd = Bt.packed_sizes()
    Xs = [synth.block_vector(A.ncols, w, synth.SEED_X + 1000 * k) for k, (A, w) in enumerate(zip(mats, widths))]
    Xd = dev(np.concatenate([v.ravel() for v in Xs]))
    Yd = torch.zeros(ny, dtype=torch.float64, device="cuda:0")
    dot = torch.zeros(nd, dtype=torch.float64, device="cuda:0")
    sc.sell_batch_spmmv_aug_packed(Bt, Xd, Yd, flags=sc.DOT_YY, dot=dot)
    Yh, dh = host(Yd), host(dot)
    yo = do = 0
    for k, (A, w) in enumerate(zip(mats, widths)):
        Yk = Yh[yo: yo + A.nrows * w].reshape(A.nrows, w)
        rows = np.unique(np.concatenate([synth.randint(90 + k, 40, 0, A.nrows - 1), [0, A.nrows - 1]]))
        _check_sampled(A, Xs[k], Yk, rows, A.val, 1e-12)
        for j in range(w):
            ref = math.fsum((Yk[:, j] * Yk[:, j]).tolist())
            assert abs(dh[3 * do + j] - ref) <= 1e-12 * ref, (k, j)
        yo += A.nrows * w
        do += w
    Bt.close()
    for M in Ms:
        M.close()
