"""GPU parity past 2^31 stored entries.

The ring matrix (synth.ring_*) of order n = 67,200,000 has 2,150,400,000 nonzeros, so entry
offsets of the SELL-C-sigma arrays pass 2^31 (row and column indices stay below it, as the
format's int32 indices require). It is generated and built on the GPU (sell_build_device),
about 27 GB of matrix. Every value and vector entry is a small dyadic rational, so every sum
of the products is exact in FP64 and FP32 in any order, and the checks are bit for bit:
sampled rows (and columns of A^T x) against the oracle on the sub-problems that hold them,
dots against sums of the GPU's own output. Sampled rows include the first and last 64 rows
and the rows stored just past offset 2^31.
"""
import numpy as np
import pytest

import synth
from gpu_util import host
from ring_util import ring_block, sample_rows, square_subproblem, transpose_subproblem

pytestmark = pytest.mark.gpu

N = 67_200_000
# With C = 32 and sigma = 1 every chunk holds a row of 34 entries, so chunk c starts at
# 34 * 32 * c: rows from 32 * ceil(2^31 / 1088) on are stored past offset 2^31.
FIRST_ROW_PAST_2_31 = 32 * -(-(2 ** 31) // (34 * 32))


@pytest.fixture(scope="module")
def sc():
    import torch

    import paper_1507_08101_amd as sc

    assert torch.cuda.is_available()
    sc.lib()
    return sc


def _say(msg):
    print(f"[large-index] {msg}", flush=True)


def _ring_matrix(sc, dtype, sigma):
    import torch

    _say(f"generate ring matrix n={N} on the GPU")
    rp, col, val = synth.ring_csr_torch(N, "cuda:0")
    _say(f"build SELL-32-{sigma} {dtype} on the GPU")
    M = sc.SellMatrix.from_device_csr(N, N, rp, col, val, C=32, sigma=sigma, dtype=dtype)
    torch.cuda.synchronize()
    del rp, col, val
    torch.cuda.empty_cache()
    return M


def _ring_dev(b, which, dtype):
    import torch

    k = torch.arange(N, dtype=torch.int64, device="cuda:0")[:, None]
    t = torch.arange(b, dtype=torch.int64, device="cuda:0")[None, :]
    v = synth.ring_x(k, t) if which == "x" else synth.ring_y(k, t)
    return v.to(dtype).contiguous()


def _rows(t, rows):
    import torch

    return host(t[torch.from_numpy(rows).to("cuda:0")])


def _exact_dots(X, Y):
    """[<y,y> | <x,y> | <x,x>] per column, FP64 sums of the GPU's own x and y (exact here)."""
    import torch

    x, y = X.double(), Y.double()
    return host(torch.cat([(y * y).sum(0), (x * y).sum(0), (x * x).sum(0)]))


AUG = dict(alpha=0.5, gamma=0.25, beta=-1.0)


def test_past_2_31_f64_sigma1(sc, orc):
    import torch

    assert synth.ring_nnz(N) > 2 ** 31
    M = _ring_matrix(sc, "f64", 1)
    info = M.info
    assert info["nnz"] == synth.ring_nnz(N)
    assert info["stored"] == 34 * N > 2 ** 31
    rows = sample_rows(N, 2048, synth.SEED_MATRIX, extra=np.arange(FIRST_ROW_PAST_2_31 - 64,
                                                                   FIRST_ROW_PAST_2_31 + 64))
    B, S, pos = square_subproblem(N, rows)

    _say("plain product, b = 1")
    X1 = _ring_dev(1, "x", torch.float64)
    Y1 = torch.zeros((N, 1), dtype=torch.float64, device="cuda:0")
    sc.sell_spmmv(M, X1, Y1)
    assert np.array_equal(_rows(Y1, rows), orc.spmmv(B, ring_block(S, 1))[pos])

    _say("augmented product with the three dots, b = 8")
    X8 = _ring_dev(8, "x", torch.float64)
    Y8 = _ring_dev(8, "y", torch.float64)
    dot = torch.zeros(24, dtype=torch.float64, device="cuda:0")
    fl = sc.SCALE | sc.SHIFT | sc.AXPBY | sc.DOT_YY | sc.DOT_XY | sc.DOT_XX
    sc.sell_spmmv_aug(M, X8, Y8, flags=fl, dot=dot, **AUG)
    ref, _, _ = orc.spmmv_aug(B, ring_block(S, 8), Y=ring_block(S, 8, "y"),
                              flags=orc.SCALE | orc.SHIFT | orc.AXPBY, **AUG)
    assert np.array_equal(_rows(Y8, rows), ref[pos])
    assert np.array_equal(host(dot), _exact_dots(X8, Y8))
    del X8, Y8

    _say("transposed product (atomic), b = 1")
    YT = torch.zeros((N, 1), dtype=torch.float64, device="cuda:0")
    sc.sell_spmmv_T(M, X1, YT, deterministic=False)
    Bt, U, Cs = transpose_subproblem(N, rows)
    assert np.array_equal(_rows(YT, Cs), orc.spmmv_T(Bt, ring_block(U, 1)))
    del YT

    _say("values-only update on the device, then b = 1")
    _, _, val1 = synth.ring_csr_torch(N, "cuda:0", variant=1, values_only=True)
    M.update_values(val1)
    torch.cuda.synchronize()
    del val1
    torch.cuda.empty_cache()
    Y1.zero_()
    sc.sell_spmmv(M, X1, Y1)
    B1, S1, pos1 = square_subproblem(N, rows, variant=1)
    assert np.array_equal(_rows(Y1, rows), orc.spmmv(B1, ring_block(S1, 1))[pos1])
    M.close()
    del X1, Y1
    torch.cuda.empty_cache()


def test_past_2_31_bf16_sigma1024_f32_vectors(sc, orc):
    import torch

    M = _ring_matrix(sc, "bf16", 1024)
    info = M.info
    assert info["nnz"] == synth.ring_nnz(N)
    assert info["has_perm"] == 1
    assert info["stored"] >= info["nnz"] > 2 ** 31
    rows = sample_rows(N, 2048, synth.SEED_Y)
    B, S, pos = square_subproblem(N, rows)

    _say("augmented product with the three dots, BF16 values, FP32 vectors, b = 8")
    X8 = _ring_dev(8, "x", torch.float32)
    Y8 = _ring_dev(8, "y", torch.float32)
    dot = torch.zeros(24, dtype=torch.float64, device="cuda:0")
    fl = sc.SCALE | sc.SHIFT | sc.AXPBY | sc.DOT_YY | sc.DOT_XY | sc.DOT_XX
    sc.sell_spmmv_aug(M, X8, Y8, flags=fl, dot=dot, **AUG)
    ref, _, _ = orc.spmmv_aug(B, ring_block(S, 8), Y=ring_block(S, 8, "y"),
                              flags=orc.SCALE | orc.SHIFT | orc.AXPBY, **AUG)
    assert np.array_equal(_rows(Y8, rows), ref[pos])
    assert np.array_equal(host(dot), _exact_dots(X8, Y8))
    M.close()
    del X8, Y8
    torch.cuda.empty_cache()
