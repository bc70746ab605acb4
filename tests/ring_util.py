"""Sub-problems of the ring matrix (synth.ring_*) that the oracle solves exactly at any order n.

A sampled output of the product y = A x, of the augmented product or of y = A^T x depends on
a few dozen rows of A and of x. These helpers cut those out as a small CSR matrix over a
renumbered index set. The oracle then computes exactly the sampled outputs of the full
problem: every value and vector entry of the ring problem is a small dyadic rational, so
every sum is exact in FP64 (and in FP32) whatever its order.
"""
import numpy as np

import synth


def _row_entries(n, rows):
    """Entries (row, position j, column) of the given sorted rows of the ring matrix."""
    offs = synth.ring_offsets(n)
    lens = synth.ring_length(rows)
    ie = np.repeat(rows, lens)
    starts = np.concatenate([[0], np.cumsum(lens)[:-1]])
    je = np.arange(int(lens.sum()), dtype=np.int64) - np.repeat(starts, lens)
    return ie, je, synth.ring_col(ie, je, offs, n), lens


def square_subproblem(n, rows, variant=0):
    """Rows R (sorted unique) of the ring matrix of order n, as a square CSR matrix over the
    index set S = R + their columns (sorted): row R[k] of A is row pos[k] of the result, with
    its columns renumbered into S; the other rows are empty. Returns (CSR, S, pos). Row pos[k]
    of an (augmented) product with x restricted to S equals row R[k] of the full product."""
    R = np.unique(np.asarray(rows, dtype=np.int64))
    ie, je, ce, lens = _row_entries(n, R)
    S = np.unique(np.concatenate([R, ce]))
    pos = np.searchsorted(S, R)
    rl = np.zeros(S.size, dtype=np.int64)
    rl[pos] = lens
    rowptr = np.zeros(S.size + 1, dtype=np.int64)
    np.cumsum(rl, out=rowptr[1:])
    col = np.searchsorted(S, ce).astype(np.int32)
    A = synth.CSR(S.size, S.size, rowptr, col, synth.ring_val(ie, je, variant), f"ring_{n}_rows")
    return A, S, pos


def transpose_subproblem(n, cols, variant=0):
    """Columns Cs (sorted unique) of the ring matrix of order n: the rows U that have an entry
    in one of them, as a CSR matrix B (len(U) x len(Cs)) holding just those entries. Returns
    (B, U, Cs); B^T x restricted to U equals y = A^T x at Cs."""
    Cs = np.unique(np.asarray(cols, dtype=np.int64))
    offs = synth.ring_offsets(n)
    j = np.arange(synth.RING_MAX_LEN, dtype=np.int64)
    cc = np.repeat(Cs, j.size)
    jj = np.tile(j, Cs.size)
    ii = (cc - offs[jj]) % n
    keep = jj < synth.ring_length(ii)
    cc, jj, ii = cc[keep], jj[keep], ii[keep]
    order = np.lexsort((cc, ii))
    cc, jj, ii = cc[order], jj[order], ii[order]
    U, inv = np.unique(ii, return_inverse=True)
    rowptr = np.zeros(U.size + 1, dtype=np.int64)
    np.cumsum(np.bincount(inv, minlength=U.size), out=rowptr[1:])
    col = np.searchsorted(Cs, cc).astype(np.int32)
    B = synth.CSR(U.size, Cs.size, rowptr, col, synth.ring_val(ii, jj, variant), f"ring_{n}_cols")
    return B, U, Cs


def ring_block(idx, b, which="x"):
    """Rows idx of the ring block vector x (or y) with b columns, FP64, row-major."""
    k = np.asarray(idx, dtype=np.int64)[:, None]
    t = np.arange(b, dtype=np.int64)[None, :]
    return (synth.ring_x(k, t) if which == "x" else synth.ring_y(k, t)).astype(np.float64)


def sample_rows(n, count, seed, extra=()):
    """Sorted unique sample: the first and last 64 rows, count seeded uniform rows, and extra."""
    r = synth.randint(seed, count, 0, n - 1).astype(np.int64)
    ends = np.concatenate([np.arange(min(64, n)), np.arange(max(0, n - 64), n)])
    return np.unique(np.concatenate([r, ends, np.asarray(extra, dtype=np.int64)]))
