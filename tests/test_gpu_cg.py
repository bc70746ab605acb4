"""GPU tests of the CG drivers: FP64 CG and BF16/FP32-value CG with FP64 iterative
refinement must reach ||b - A x|| <= 1e-10 ||b||, with the residual recomputed by the
CPU oracle from the returned x."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, host

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def sc():
    import torch

    import paper_1507_08101_amd as sc

    assert torch.cuda.is_available()
    sc.lib()
    return sc


def _true_relres(A, B, X):
    R = B - oracle.spmmv(A, X)
    return np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0)


@pytest.mark.parametrize("b", [1, 3, 8])
def test_cg_fp64_reaches_tolerance(sc, b):
    A = synth.laplacian3d(24)
    B = synth.block_vector(A.nrows, b, synth.SEED_Y)
    M = sc.SellMatrix.from_csr(A, C=32, sigma=1)
    Xd = dev(np.zeros_like(B))
    st = sc.sell_cg(M, dev(B), Xd, tol=TOL)
    X = host(Xd)
    rr = _true_relres(A, B, X)
    assert st["converged"] == 1 and rr.max() <= TOL * 1.001, (st, rr)
    assert abs(st["relres"] - rr.max()) <= 1e-3 * rr.max() + 1e-14
    # the same solution the oracle's CG reaches, to within the conditioning
    lmin = 6 - 6 * math.cos(math.pi / 25)
    for j in range(b):
        xo, _ = oracle.cg(A, B[:, j], tol=TOL)
        assert np.linalg.norm(X[:, j] - xo) <= 2 * TOL * np.linalg.norm(B[:, j]) / lmin
    M.close()


# The iteration's vector pass runs on 16-byte column groups when b is a multiple of the
# group (2 doubles, 4 floats) with a power-of-two number of groups per row up to 16, and per
# element otherwise: every group count and both fallbacks (3 groups; 32 groups).
@pytest.mark.parametrize("b", [2, 4, 6, 8, 16, 32, 64])
def test_cg_fp64_every_vector_pass_width(sc, b):
    A = synth.laplacian3d(9)
    B = synth.block_vector(A.nrows, b, 40 + b)
    M = sc.SellMatrix.from_csr(A, C=32, sigma=1)
    Xd = dev(np.zeros_like(B))
    st = sc.sell_cg(M, dev(B), Xd, tol=TOL)
    rr = _true_relres(A, B, host(Xd))
    assert st["converged"] == 1 and rr.max() <= TOL * 1.001, (b, st, rr)
    M.close()


@pytest.mark.parametrize("b", [3, 4, 8, 12, 16, 32, 64])
def test_cg_mixed_every_vector_pass_width(sc, b):
    A = synth.laplacian3d(9)
    B = synth.block_vector(A.nrows, b, 60 + b)
    A64 = sc.SellMatrix.from_csr(A, C=32, sigma=1)
    Alo = sc.SellMatrix.from_csr(A, C=32, sigma=1, dtype="bf16")
    Xd = dev(np.zeros_like(B))
    st = sc.sell_cg_mixed(A64, Alo, dev(B), Xd, tol=TOL)
    rr = _true_relres(A, B, host(Xd))
    assert st["converged"] == 1 and rr.max() <= TOL * 1.001, (b, st, rr)
    A64.close()
    Alo.close()


def test_cg_fp64_unaligned_solution_takes_the_element_pass(sc):
    """x 8 bytes past a 16-byte boundary sends the vector pass (which updates x) to the
    per-element kernel: the solve agrees with the aligned one (column groups) to the tolerance
    and in its iteration count (only the rounding of the dots differs)."""
    import torch

    A = synth.laplacian3d(12)
    b = 8
    B = synth.block_vector(A.nrows, b, 77)
    M = sc.SellMatrix.from_csr(A, C=32, sigma=1)
    out = []
    for off in (0, 1):
        buf = torch.zeros(A.nrows * b + 2, dtype=torch.float64, device="cuda:0")
        Xd = buf[off:off + A.nrows * b].view(A.nrows, b)
        assert (Xd.data_ptr() % 16 == 0) == (off == 0)
        st = sc.sell_cg(M, dev(B), Xd, tol=TOL)
        X = host(Xd)
        rr = _true_relres(A, B, X)
        assert st["converged"] == 1 and rr.max() <= TOL * 1.001, (off, st, rr)
        out.append((X, st["iterations"]))
    assert abs(out[0][1] - out[1][1]) <= 2
    lmin = 6 - 6 * math.cos(math.pi / 13)
    for j in range(b):
        assert np.linalg.norm(out[0][0][:, j] - out[1][0][:, j]) <= 4 * TOL * np.linalg.norm(B[:, j]) / lmin
    M.close()


@pytest.mark.parametrize("lo", ["bf16", "f32"])
def test_cg_mixed_reaches_tolerance(sc, lo):
    A = synth.laplacian3d(24)
    b = 8
    B = synth.block_vector(A.nrows, b, synth.SEED_Y)
    A64 = sc.SellMatrix.from_csr(A, C=32, sigma=1)
    Alo = sc.SellMatrix.from_csr(A, C=32, sigma=1, dtype=lo)
    Xd = dev(np.zeros_like(B))
    st = sc.sell_cg_mixed(A64, Alo, dev(B), Xd, tol=TOL)
    X = host(Xd)
    rr = _true_relres(A, B, X)
    assert st["converged"] == 1 and rr.max() <= TOL * 1.001, (st, rr)
    assert st["refinements"] >= 2  # one FP32 solve alone cannot reach 1e-10
    A64.close()
    Alo.close()


def test_cg_mixed_on_matrix_not_exact_in_bf16(sc):
    # an SPD matrix whose values are not bf16 numbers: the low-precision operator differs
    # from A, refinement still converges to the FP64 tolerance
    L = synth.laplacian3d(16)
    shift = synth.uniform(9, L.nrows, 0.3, 0.7)
    val = L.val.copy()
    rows = np.repeat(np.arange(L.nrows), L.row_lengths())
    diag = L.col == rows
    val[diag] += shift
    val[~diag] *= 1.0 + 0.01 * synth.uniform(10, int((~diag).sum()), -1, 1)
    # keep it symmetric: average with the transpose
    import scipy.sparse as sp

    S = sp.csr_matrix((val, L.col, L.rowptr), shape=(L.nrows, L.nrows))
    S = ((S + S.T) * 0.5).tocsr()
    S.sort_indices()
    A = synth.CSR(L.nrows, L.nrows, S.indptr, S.indices, S.data, "spd")
    assert not np.array_equal(oracle.round_bf16(A.val), A.val)
    b = 4
    B = synth.block_vector(A.nrows, b, 11)
    A64 = sc.SellMatrix.from_csr(A, C=32, sigma=64)
    Alo = sc.SellMatrix.from_csr(A, C=32, sigma=64, dtype="bf16")
    Xd = dev(np.zeros_like(B))
    st = sc.sell_cg_mixed(A64, Alo, dev(B), Xd, tol=TOL)
    rr = _true_relres(A, B, host(Xd))
    assert st["converged"] == 1 and rr.max() <= TOL * 1.001, (st, rr)
    A64.close()
    Alo.close()


@pytest.mark.parametrize("e", [2, 3, 5])
@pytest.mark.parametrize("lo", ["bf16", "f32"])
def test_cg_mixed_small_systems(sc, e, lo):
    """FP32 CG exhausts a system of e^3 unknowns within a few checks: its recursive residual
    falls far below the true one, and the refinement must restart those columns from p = r
    rather than keep a direction of vanishing size."""
    A = synth.laplacian3d(e)
    b = 4
    B = synth.block_vector(A.nrows, b, 12 + e)
    A64 = sc.SellMatrix.from_csr(A, C=32, sigma=1)
    Alo = sc.SellMatrix.from_csr(A, C=32, sigma=1, dtype=lo)
    Xd = dev(np.zeros_like(B))
    st = sc.sell_cg_mixed(A64, Alo, dev(B), Xd, tol=TOL, maxit=2000)
    rr = _true_relres(A, B, host(Xd))
    assert st["converged"] == 1 and rr.max() <= TOL * 1.001, (st, rr)
    assert st["iterations"] < 400, st
    A64.close()
    Alo.close()


def test_cg_rejects_bad_operands(sc):
    import torch

    A = synth.laplacian3d(6)
    M = sc.SellMatrix.from_csr(A, C=32, sigma=1)
    B = torch.zeros((A.nrows, 2), dtype=torch.float32, device="cuda:0")
    X = torch.zeros((A.nrows, 2), dtype=torch.float32, device="cuda:0")
    with pytest.raises(sc.SellError) as e:
        sc.sell_cg(M, B, X)
    assert e.value.code == sc.SELL_ERR_DTYPE
    with pytest.raises(sc.SellError) as e:
        sc.sell_cg_mixed(M, M, B.double(), X.double())
    assert e.value.code == sc.SELL_ERR_DTYPE
    M.close()
