"""GPU tests of differentiation with respect to the stored matrix values: the pattern-
restricted outer product, the single-product autograd function (torch.autograd.gradcheck,
i.e. central finite differences in FP64, runs the HIP kernels), and the Chebyshev
application T_N(A(theta)) x with recompute checkpoints against the oracle's FP64 adjoint and
against finite differences."""
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


def _relnorm(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("b", [1, 3, 8])
def test_grad_values_matches_oracle(sc, b):
    import torch

    A = synth.random_sparse(300, 170, 0.05, 120, duplicates=True, empty_rows=7)
    M = sc.SellMatrix.from_csr(A, C=32, sigma=64)
    G = synth.block_vector(A.nrows, b, 121)
    X = synth.block_vector(A.ncols, b, 122)
    dval = torch.full((A.nnz,), 5.0, dtype=torch.float64, device="cuda:0")
    sc.sell_grad_values(M, dev(G), dev(X), dval, alpha=2.0)
    ref = 2.0 * oracle.pattern_outer(A, G, X)
    assert _relnorm(host(dval), ref) <= 1e-14
    sc.sell_grad_values(M, dev(G), dev(X), dval, alpha=1.0, accumulate=True)
    assert _relnorm(host(dval), 1.5 * ref) <= 1e-14
    M.close()


def test_spmm_autograd_gradcheck(sc):
    import torch

    from paper_1507_08101_amd.autograd import spmm

    A = synth.random_sparse(40, 30, 0.15, 123)
    M = sc.SellMatrix.from_csr(A, C=8, sigma=16)
    theta = torch.tensor(A.val, dtype=torch.float64, device="cuda:0", requires_grad=True)
    X = torch.tensor(synth.block_vector(30, 2, 124), device="cuda:0", requires_grad=True)
    assert torch.autograd.gradcheck(lambda t, x: spmm(t, x, M), (theta, X), eps=1e-6, atol=1e-8, rtol=1e-6)
    M.close()


def test_transpose_follows_value_updates(sc):
    import torch

    A = synth.random_sparse(120, 90, 0.06, 125)
    M = sc.SellMatrix.from_csr(A, C=32, sigma=32)
    X = synth.block_vector(A.nrows, 2, 126)
    Y = torch.zeros((A.ncols, 2), dtype=torch.float64, device="cuda:0")
    sc.sell_spmmv_T(M, dev(X), Y, deterministic=True)  # builds the copy of A^T
    newv = synth.uniform(127, A.nnz, -2, 2)
    M.update_values(dev(newv))
    sc.sell_spmmv_T(M, dev(X), Y, deterministic=True)
    A2 = synth.CSR(A.nrows, A.ncols, A.rowptr, A.col, newv)
    assert _relnorm(host(Y), oracle.spmmv_T(A2, X)) <= 1e-14
    M.close()


def test_first_transpose_after_update_on_side_stream(sc):
    """A value update queued on a non-blocking side stream, then the first deterministic
    transposed product on that stream: the copy of A^T it builds must hold the new values."""
    import torch

    A = synth.random_sparse(2000, 1500, 0.01, 128)
    M = sc.SellMatrix.from_csr(A, C=32, sigma=64)
    X = synth.block_vector(A.nrows, 3, 129)
    newv = synth.uniform(130, A.nnz, -2, 2)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        nv = dev(newv)
        Xd = dev(X)
        side.synchronize()
        # a long kernel queued first keeps the stream busy while the update waits behind it
        big = torch.randn(4096, 4096, dtype=torch.float64, device="cuda:0")
        for _ in range(4):
            big = big @ big * 1e-3
        M.update_values(nv)  # on the current stream: side
        Y = torch.zeros((A.ncols, 3), dtype=torch.float64, device="cuda:0")
        sc.sell_spmmv_T(M, Xd, Y, deterministic=True)
    side.synchronize()
    A2 = synth.CSR(A.nrows, A.ncols, A.rowptr, A.col, newv)
    assert _relnorm(host(Y), oracle.spmmv_T(A2, X)) <= 1e-14
    M.close()


@pytest.mark.parametrize("fn", ["spmm", "chebyshev"])
def test_autograd_two_forwards_one_handle(sc, fn):
    """Two forwards with different theta on one matrix handle before either backward: each
    backward must give the gradients of the matrix its own forward used."""
    import torch

    from paper_1507_08101_amd.autograd import chebyshev, spmm

    A = synth.anderson3d(6)
    s = (6 + 16.5 / 2) / 0.99
    M = sc.SellMatrix.from_csr(A, C=32, sigma=1)
    X = synth.block_vector(A.nrows, 2, 131)
    th1 = A.val.copy()
    th2 = A.val * synth.uniform(132, A.nnz, 0.5, 1.0)
    run = (lambda t, x: spmm(t, x, M)) if fn == "spmm" else (lambda t, x: chebyshev(t, x, M, 7, s, 0.0, 3))
    grads = []
    outs = []
    for th in (th1, th2):
        t = torch.tensor(th, device="cuda:0", requires_grad=True)
        x = torch.tensor(X, device="cuda:0", requires_grad=True)
        outs.append((t, x, run(t, x)))
    for t, x, y in reversed(outs):  # backward of the second forward first, then the first
        (y * y).sum().backward()
        grads.append((host(t.grad), host(x.grad)))
    grads.reverse()
    for (th, (gt, gx)) in zip((th1, th2), grads):
        Ak = synth.CSR(A.nrows, A.ncols, A.rowptr, A.col, th)
        if fn == "spmm":
            Y = oracle.spmmv(Ak, X)
            rx, rt = oracle.spmmv_T(Ak, 2 * Y), oracle.pattern_outer(Ak, 2 * Y, X)
        else:
            Y = oracle.cheb_apply(Ak, X, 7, s, 0.0)
            rx, rt = oracle.cheb_grad(Ak, X, 7, s, 0.0, 2 * Y)
        assert _relnorm(gx, rx) <= 1e-12 and _relnorm(gt, rt) <= 1e-12
    M.close()


def _anderson_case(L, b, seed):
    A = synth.anderson3d(L)
    s = (6 + 16.5 / 2) / 0.99
    X = synth.block_vector(A.nrows, b, seed)
    return A, s, X


@pytest.mark.parametrize("N,K,b", [(1, 10, 1), (7, 3, 2), (20, 6, 1), (20, 20, 3), (20, 40, 1)])
def test_chebyshev_forward_backward_vs_oracle(sc, N, K, b):
    import torch

    from paper_1507_08101_amd.autograd import chebyshev

    A, s, X = _anderson_case(10, b, 130)
    c = 0.3
    M = sc.SellMatrix.from_csr(A, C=32, sigma=1)
    theta = torch.tensor(A.val, dtype=torch.float64, device="cuda:0", requires_grad=True)
    Xd = torch.tensor(X, device="cuda:0", requires_grad=True)
    Y = chebyshev(theta, Xd, M, N, s, c, K)
    Yref = oracle.cheb_apply(A, X, N, s, c)
    assert _relnorm(host(Y), Yref) <= 1e-12
    loss = (Y * Y).sum()
    loss.backward()
    dX_ref, dval_ref = oracle.cheb_grad(A, X, N, s, c, 2.0 * Yref)
    assert _relnorm(host(Xd.grad), dX_ref) <= 1e-11
    assert _relnorm(host(theta.grad), dval_ref) <= 1e-11
    M.close()


def test_chebyshev_general_nonsymmetric(sc):
    # a nonsymmetric matrix exercises the A^T path of the adjoint
    import torch

    from paper_1507_08101_amd.autograd import chebyshev

    A = synth.random_sparse(500, 500, 0.01, 131, empty_rows=4)
    s, c, N, K = 3.0, 0.1, 9, 4
    X = synth.block_vector(500, 2, 132)
    W = synth.block_vector(500, 2, 133)
    M = sc.SellMatrix.from_csr(A, C=16, sigma=50)
    theta = torch.tensor(A.val, dtype=torch.float64, device="cuda:0", requires_grad=True)
    Xd = torch.tensor(X, device="cuda:0", requires_grad=True)
    Y = chebyshev(theta, Xd, M, N, s, c, K)
    (Y * dev(W)).sum().backward()
    dX_ref, dval_ref = oracle.cheb_grad(A, X, N, s, c, W)
    assert _relnorm(host(Xd.grad), dX_ref) <= 1e-11
    assert _relnorm(host(theta.grad), dval_ref) <= 1e-11
    M.close()


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_chebyshev_degree100_anderson64(sc, dt):
    """The differentiation workload: T_100 of the 64^3 Anderson matrix, loss sum(y^2),
    checkpoints every 10 steps; FP64 against the oracle's FP64 adjoint, FP32 against the
    oracle's adjoint of the float32-rounded values, and FP64 against central differences."""
    import torch

    from paper_1507_08101_amd.autograd import chebyshev

    A, s, X = _anderson_case(64, 1, 140)
    N, K = 100, 10
    M = sc.SellMatrix.from_csr(A, C=32, sigma=1, dtype=dt)
    vt = torch.float64 if dt == "f64" else torch.float32
    Xin = X if dt == "f64" else X.astype(np.float32).astype(np.float64)
    theta = torch.tensor(A.val, dtype=torch.float64, device="cuda:0", requires_grad=True)
    Xd = torch.tensor(Xin, dtype=vt, device="cuda:0", requires_grad=True)
    Y = chebyshev(theta, Xd, M, N, s, 0.0, K)
    loss = (Y.double() ** 2).sum()
    loss.backward()
    Ar = A if dt == "f64" else synth.CSR(A.nrows, A.ncols, A.rowptr, A.col, oracle.round_f32(A.val))
    Yref = oracle.cheb_apply(Ar, Xin, N, s)
    dX_ref, dval_ref = oracle.cheb_grad(Ar, Xin, N, s, 0.0, 2.0 * Yref)
    tol = 1e-10 if dt == "f64" else 2e-4
    assert _relnorm(host(Y), Yref) <= tol
    assert _relnorm(host(Xd.grad), dX_ref) <= tol
    assert _relnorm(host(theta.grad), dval_ref) <= tol
    if dt == "f64":
        # central differences on a few values, through the GPU forward pass
        g = host(theta.grad)
        h = 1e-6
        for p in [0, 1234567 % A.nnz, A.nnz - 1, int(np.argmax(np.abs(g)))]:
            ys = []
            for sgn in (1, -1):
                th = torch.tensor(A.val, dtype=torch.float64, device="cuda:0")
                th[p] += sgn * h
                with torch.no_grad():
                    ys.append(host(chebyshev(th, torch.tensor(X, device="cuda:0"), M, N, s, 0.0, K)))
            # L(+h) - L(-h) = sum (y+ - y-)(y+ + y-): no cancellation between two large sums
            fd = float(np.sum((ys[0] - ys[1]) * (ys[0] + ys[1]))) / (2 * h)
            assert abs(fd - g[p]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), p
    M.close()
