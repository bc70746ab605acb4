"""The ring matrix inputs (synth.ring_*) and their sampled sub-problems, on the CPU.

The GPU test past 2^31 stored entries relies on three facts checked here at a size the oracle
handles whole: the closed-form nonzero count, the host and torch generators agreeing entry for
entry, and the sub-problems reproducing the full product's sampled rows (and columns of A^T x)
bit for bit, which holds because every sum of the ring problem is exact in FP64 and FP32.
"""
import numpy as np
import pytest

import synth
from ring_util import ring_block, sample_rows, square_subproblem, transpose_subproblem

N = 300_007  # n mod 5 = 2, n mod 32 = 23: a ragged last chunk


@pytest.fixture(scope="module")
def ring():
    return synth.ring_csr(N)


@pytest.mark.parametrize("n", [1 << 19, 300_007, 1_000_003, 67_200_000])
def test_ring_nnz_closed_form_and_offsets(n):
    lens = synth.ring_length(np.arange(n, dtype=np.int64))
    assert int(lens.sum()) == synth.ring_nnz(n)
    assert lens.min() == 30 and lens.max() == synth.RING_MAX_LEN
    offs = synth.ring_offsets(n)
    assert len(set((offs % n).tolist())) == synth.RING_MAX_LEN
    assert np.all(np.abs(offs) < n // 2)


def test_ring_large_order_passes_2_31():
    # the order used on the GPU: 2,150,400,000 nonzeros > 2^31
    assert synth.ring_nnz(67_200_000) == 2_150_400_000 > 2 ** 31
    for small in (1000, 1 << 18):  # n / 64 = 4096 collides with a short offset at 2^18
        with pytest.raises(ValueError):
            synth.ring_offsets(small)


def test_ring_pattern_and_values(ring):
    A = ring
    assert A.nnz == synth.ring_nnz(N)
    assert A.col.min() >= 0 and A.col.max() < N
    for i in [0, 1, 4, 12345, N - 1]:
        c = A.col[A.rowptr[i]:A.rowptr[i + 1]]
        assert c.size == 30 + i % 5 and np.unique(c).size == c.size
    v4 = A.val * 4
    assert np.array_equal(v4, np.rint(v4)) and np.all(np.abs(v4) >= 1) and np.all(np.abs(v4) <= 7)
    x = ring_block(np.arange(100), 8) * 8
    assert np.array_equal(x, np.rint(x)) and np.abs(x).max() <= 8


def test_ring_torch_generator_matches_host(ring):
    torch = pytest.importorskip("torch")
    rp, col, val = synth.ring_csr_torch(N, "cpu", chunk_rows=65_536)
    assert np.array_equal(rp.numpy(), ring.rowptr)
    assert np.array_equal(col.numpy(), ring.col)
    assert np.array_equal(val.numpy(), ring.val)
    _, none, v1 = synth.ring_csr_torch(N, "cpu", variant=1, chunk_rows=100_000, values_only=True)
    assert none is None
    assert np.array_equal(v1.numpy(), synth.ring_csr(N, variant=1).val)
    assert not np.array_equal(v1.numpy(), ring.val)
    assert torch.all(rp[1:] >= rp[:-1])


def test_square_subproblem_reproduces_full_rows(orc, ring):
    rows = sample_rows(N, 300, synth.SEED_MATRIX, extra=[N // 2])
    X = ring_block(np.arange(N), 8)
    Y0 = ring_block(np.arange(N), 8, "y")
    full = orc.spmmv(ring, X)
    flags = orc.SCALE | orc.SHIFT | orc.AXPBY
    full_aug, _, _ = orc.spmmv_aug(ring, X, Y=Y0, flags=flags, alpha=0.5, gamma=0.25, beta=-1.0)
    B, S, pos = square_subproblem(N, rows)
    sub = orc.spmmv(B, ring_block(S, 8))
    sub_aug, _, _ = orc.spmmv_aug(B, ring_block(S, 8), Y=ring_block(S, 8, "y"), flags=flags, alpha=0.5,
                                  gamma=0.25, beta=-1.0)
    assert np.array_equal(sub[pos], full[rows])
    assert np.array_equal(sub_aug[pos], full_aug[rows])
    # exactness: every row's entries in the opposite order give the same bits
    lens = np.diff(ring.rowptr)
    starts = np.repeat(ring.rowptr[:-1], lens)
    j = np.arange(ring.nnz) - starts
    src = starts + np.repeat(lens, lens) - 1 - j
    rev = synth.CSR(ring.nrows, ring.ncols, ring.rowptr, ring.col[src], ring.val[src])
    assert not np.array_equal(rev.col, ring.col)
    assert np.array_equal(orc.spmmv(rev, X), full)


def test_transpose_subproblem_reproduces_full_columns(orc, ring):
    cols = sample_rows(N, 300, synth.SEED_X)
    x = ring_block(np.arange(N), 1)
    full = orc.spmmv_T(ring, x)
    B, U, Cs = transpose_subproblem(N, cols)
    assert np.array_equal(Cs, cols)
    sub = orc.spmmv_T(B, ring_block(U, 1))
    assert np.array_equal(sub, full[cols])
    # every column of the ring matrix holds one entry per offset whose row is long enough
    colcount = np.bincount(ring.col, minlength=N)
    assert np.array_equal(np.bincount(B.col, minlength=Cs.size), colcount[Cs])
