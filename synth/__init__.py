"""Seeded synthetic inputs shaped like the GHOST paper's workloads.

This module only *makes inputs*: CSR matrices (row pointers int64, column
indices int32, values float64, columns sorted and unique within a row) and
dense block vectors. It holds none of the sparse-product arithmetic, so both
the CPU oracle and the HIP library can take their inputs from here without
sharing any of the method.

Random numbers come from a counter-based SplitMix64 stream (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014; the
finaliser constants are the published ones): element ``i`` of stream
``seed`` is ``mix(seed + (i + 1) * 0x9E3779B97F4A7C15)``.  Uniform doubles use
the top 53 bits; normals use the Box-Muller transform.  Fixed seeds make every
run reproducible, as the paper asks of its own random inputs (Sec. 6.1).

Workload shapes (the paper's test matrices are not available, so these stand
in for them; the sizes come from the workload definitions this project
measures):

* ``laplacian2d(N)``   2D 5-point Dirichlet Laplacian, values 4 / -1.
* ``laplacian3d(e)``   3D 7-point Dirichlet Laplacian, values 6 / -1 (SPD).
* ``anderson3d(L)``    3D periodic Anderson Hamiltonian: hopping -1, on-site
                       disorder U[-W/2, W/2] with W = 16.5.
* ``irregular(n)``     lognormal row lengths (mean 15, clipped to [1, 2000]);
                       half of each row's columns in a +-5000 band around the
                       diagonal (reflected at the borders), half uniform;
                       values N(0, 1).
* ``ring_*``           a matrix given entry by entry by formulas, for sizes past
                       2^31 stored entries: row i has 30 + i mod 5 entries, entry
                       j at column (i + offset_j) mod n, with small dyadic values;
                       block vectors by formula as well. Its columns keep the
                       offsets' order (unique within a row, not sorted). The
                       formulas work on numpy arrays and torch tensors alike, so
                       the same matrix can be made on the host and on a GPU.
"""
from __future__ import annotations

import math

import numpy as np

SEED_MATRIX = 150708101
SEED_X = 150708102
SEED_Y = 150708103

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def substream(seed: int, tag: int) -> int:
    """Derive an independent stream seed from ``seed`` and a small tag."""
    z = np.array([(seed * 0x100000001B3 + tag * 0x9E3779B97F4A7C15) % (1 << 64)], dtype=np.uint64)
    return int(_mix(z)[0])


def bits(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """``count`` 64-bit outputs of the counter-based SplitMix64 stream ``seed``."""
    ctr = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        x = np.uint64(seed % (1 << 64)) + ctr * _GOLDEN
    return _mix(x)


def uniform01(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits."""
    return (bits(seed, count, offset) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform(seed: int, count: int, lo: float, hi: float, offset: int = 0) -> np.ndarray:
    return lo + (hi - lo) * uniform01(seed, count, offset)


def randint(seed: int, count: int, lo: int, hi: int, offset: int = 0) -> np.ndarray:
    """Integers uniform on [lo, hi] (inclusive) by multiply-shift of the top 32 bits."""
    span = hi - lo + 1
    assert 0 < span <= (1 << 32)
    top = bits(seed, count, offset) >> np.uint64(32)
    with np.errstate(over="ignore"):
        r = (top * np.uint64(span)) >> np.uint64(32)
    return lo + r.astype(np.int64)


def normal(seed: int, count: int) -> np.ndarray:
    """Standard normals by Box-Muller (cosine branch only)."""
    u1 = 1.0 - uniform01(substream(seed, 1), count)  # (0, 1]
    u2 = uniform01(substream(seed, 2), count)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


# --------------------------------------------------------------------------------------
# block vectors


def block_vector(n: int, b: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Row-major n x b block vector with entries U[lo, hi]."""
    return uniform(seed, n * b, lo, hi).reshape(n, b)


def int_block_vector(n: int, b: int, seed: int, lo: int = -8, hi: int = 8) -> np.ndarray:
    """Row-major n x b block vector of small integers (exact in every precision used)."""
    return randint(seed, n * b, lo, hi).astype(np.float64).reshape(n, b)


# --------------------------------------------------------------------------------------
# matrices


class CSR:
    """A plain CSR matrix: rowptr int64[n+1], col int32[nnz], val float64[nnz]."""

    def __init__(self, nrows: int, ncols: int, rowptr, col, val, name: str = ""):
        self.nrows = int(nrows)
        self.ncols = int(ncols)
        self.rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)
        self.name = name
        assert self.rowptr.shape == (self.nrows + 1,)
        assert self.col.shape == self.val.shape == (int(self.rowptr[-1]),)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.rowptr)

    def dense(self) -> np.ndarray:
        """Dense copy (small matrices only). Duplicate entries are summed."""
        d = np.zeros((self.nrows, self.ncols))
        rows = np.repeat(np.arange(self.nrows), self.row_lengths())
        np.add.at(d, (rows, self.col.astype(np.int64)), self.val)
        return d

    def __repr__(self) -> str:
        return f"CSR({self.name!r}, n={self.nrows}x{self.ncols}, nnz={self.nnz})"


def _from_coo(n: int, m: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray, name: str) -> CSR:
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    return CSR(n, m, rowptr, cols.astype(np.int32), vals, name)


def _stencil(dims, periodic: bool, diag: np.ndarray, off: float, name: str) -> CSR:
    """Nearest-neighbour stencil on a lexicographically ordered grid (x fastest)."""
    dims = tuple(int(d) for d in dims)
    n = int(np.prod(dims))
    idx = np.arange(n, dtype=np.int64)
    coords = []
    rem = idx.copy()
    for d in dims:
        coords.append(rem % d)
        rem //= d
    strides = [int(np.prod(dims[:k])) for k in range(len(dims))]
    rows = [idx]
    cols = [idx]
    vals = [np.asarray(diag, dtype=np.float64)]
    for k, d in enumerate(dims):
        for step in (-1, 1):
            c = coords[k] + step
            if periodic:
                if d < 3:
                    raise ValueError("periodic stencil needs at least 3 points per dimension")
                wrapped = c % d
                rows.append(idx)
                cols.append(idx + (wrapped - coords[k]) * strides[k])
                vals.append(np.full(n, off))
            else:
                ok = (c >= 0) & (c < d)
                rows.append(idx[ok])
                cols.append(idx[ok] + step * strides[k])
                vals.append(np.full(int(ok.sum()), off))
    return _from_coo(n, n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), name)


def laplacian2d(N: int) -> CSR:
    """2D 5-point Dirichlet Laplacian on an N x N grid (4 on the diagonal, -1 off it)."""
    n = N * N
    return _stencil((N, N), False, np.full(n, 4.0), -1.0, f"lap2d_{N}")


def laplacian3d(e: int) -> CSR:
    """3D 7-point Dirichlet Laplacian on an e^3 grid (6 / -1); symmetric positive definite."""
    n = e ** 3
    return _stencil((e, e, e), False, np.full(n, 6.0), -1.0, f"lap3d_{e}")


def anderson3d(L: int, W: float = 16.5, seed: int = SEED_MATRIX) -> CSR:
    """3D periodic Anderson Hamiltonian on an L^3 lattice: hopping -1, disorder U[-W/2, W/2]."""
    n = L ** 3
    eps = uniform(substream(seed, 7), n, -W / 2.0, W / 2.0)
    return _stencil((L, L, L), True, eps, -1.0, f"anderson3d_{L}")


def irregular(n: int, mean_len: float = 15.0, sigma_ln: float = 1.0, max_len: int = 2000,
              band: int = 5000, seed: int = SEED_MATRIX) -> CSR:
    """Irregular matrix with lognormal row lengths; half banded, half uniform columns.

    Row length = clip(rint(exp(mu + sigma_ln * z)), 1, min(max_len, n)) with
    mu = ln(mean_len) - sigma_ln^2 / 2.  The first ceil(len/2) columns of a row are
    i + U{-band..band} reflected into [0, n); the rest are U{0..n-1}.  Duplicates in
    a row are re-drawn uniformly until none remain; columns are then sorted.
    """
    mu = math.log(mean_len) - 0.5 * sigma_ln * sigma_ln
    z = normal(substream(seed, 11), n)
    lens = np.clip(np.rint(np.exp(mu + sigma_ln * z)), 1, min(max_len, n)).astype(np.int64)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=rowptr[1:])
    nnz = int(rowptr[-1])
    rows = np.repeat(np.arange(n, dtype=np.int64), lens)
    pos = np.arange(nnz, dtype=np.int64) - rowptr[rows]
    in_band = pos < (lens[rows] + 1) // 2
    bw = min(band, max(n - 1, 0))
    off = randint(substream(seed, 12), nnz, -bw, bw) if bw > 0 else np.zeros(nnz, np.int64)
    cb = rows + off
    cb = np.where(cb < 0, -cb, cb)
    cb = np.where(cb >= n, 2 * (n - 1) - cb, cb)
    cu = randint(substream(seed, 13), nnz, 0, n - 1)
    cols = np.where(in_band, cb, cu)
    rnd = 0
    while True:
        key = rows * n + cols
        order = np.argsort(key, kind="stable")
        key = key[order]
        cols = cols[order]
        dup = np.zeros(nnz, dtype=bool)
        dup[1:] = key[1:] == key[:-1]
        ndup = int(dup.sum())
        if ndup == 0:
            break
        rnd += 1
        cols[dup] = randint(substream(seed, 100 + rnd), ndup, 0, n - 1)
    vals = normal(substream(seed, 14), nnz)
    return CSR(n, n, rowptr, cols.astype(np.int32), vals, f"irregular_{n}")


def random_sparse(nrows: int, ncols: int, density: float, seed: int, int_values: bool = False,
                  empty_rows: int = 0, long_row: int = 0, duplicates: bool = False) -> CSR:
    """Small random pattern for tests: Bernoulli(density) entries, optional empty rows,
    one optional long row, optional duplicated entries (kept as separate entries)."""
    u = uniform01(substream(seed, 21), nrows * ncols).reshape(nrows, ncols)
    mask = u < density
    if empty_rows:
        er = randint(substream(seed, 22), empty_rows, 0, nrows - 1)
        mask[er, :] = False
    if long_row and nrows > 0:
        r = int(randint(substream(seed, 23), 1, 0, nrows - 1)[0])
        mask[r, : min(long_row, ncols)] = True
    rows, cols = np.nonzero(mask)
    if int_values:
        vals = randint(substream(seed, 24), rows.size, -4, 4).astype(np.float64)
    else:
        vals = uniform(substream(seed, 24), rows.size, -1.0, 1.0)
    if duplicates and rows.size:
        pick = randint(substream(seed, 25), max(1, rows.size // 10), 0, rows.size - 1)
        rows = np.concatenate([rows, rows[pick]])
        cols = np.concatenate([cols, cols[pick]])
        extra = uniform(substream(seed, 26), pick.size, -1.0, 1.0)
        if int_values:
            extra = np.rint(4 * extra)
        vals = np.concatenate([vals, extra])
        # keep the extra copies next to their originals, original first
        order = np.lexsort((np.arange(rows.size), cols, rows))
        rows, cols, vals = rows[order], cols[order], vals[order]
        rowptr = np.zeros(nrows + 1, dtype=np.int64)
        np.cumsum(np.bincount(rows, minlength=nrows), out=rowptr[1:])
        return CSR(nrows, ncols, rowptr, cols.astype(np.int32), vals, f"random_dup_{nrows}x{ncols}")
    rowptr = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=nrows), out=rowptr[1:])
    return CSR(nrows, ncols, rowptr, cols.astype(np.int32), vals, f"random_{nrows}x{ncols}")


def laplacian3d_batch(count: int = 64, lo: int = 20, hi: int = 100, seed: int = SEED_MATRIX):
    """Grid edges for a batch of 3D Laplacians, edge ~ U{lo..hi}, one per matrix."""
    return [int(e) for e in randint(substream(seed, 31), count, lo, hi)]


# --------------------------------------------------------------------------------------
# formula ("ring") matrices: sizes past 2^31 stored entries without random streams


RING_MAX_LEN = 34


def ring_offsets(n: int) -> np.ndarray:
    """The 34 column offsets of the ring matrix of order n, distinct modulo n (n >= 2^19):
    short ones (neighbours, rows of a 64-wide grid), and fractions of n up to n/2 (far gathers)."""
    near = [1, 2, 3, 5, 64, 65, 4096, 4097]
    far = [n // 64, n // 64 + 1, n // 16, n // 16 + 3, n // 8, n // 5, n // 3, n // 3 + 7, n // 2 - 1]
    offs = [0, *[s * o for o in near + far for s in (1, -1)]][:RING_MAX_LEN]
    out = np.array(offs, dtype=np.int64)
    if len(out) != RING_MAX_LEN or len(set((out % n).tolist())) != RING_MAX_LEN:
        raise ValueError(f"ring offsets not distinct modulo n = {n}")
    return out


def ring_length(i):
    """Entries of row i (numpy array or torch tensor of int64 rows): 30 + i mod 5."""
    return 30 + i % 5


def ring_nnz(n: int) -> int:
    """Closed form of sum_{i < n} (30 + i mod 5)."""
    r = n % 5
    return 30 * n + 10 * (n // 5) + r * (r - 1) // 2


def ring_col(i, j, offs, n: int):
    """Column of entry j of row i: (i + offs[j]) mod n (offs indexable by j: a numpy array for
    numpy j, a tensor on j's device for torch j)."""
    return (i + offs[j]) % n


def ring_val(i, j, variant: int = 0):
    """Value of entry j of row i: +-m / 4 with m in 1..7 (exact in BF16, FP32 and FP64).
    variant 1 gives a second set of values on the same pattern."""
    a, c = (5, 3) if variant == 0 else (3, 5)
    mag = (a * i + c * j) % 7 + 1
    sign = 1 - 2 * ((i + j + variant) % 2)
    return (mag * sign) * 0.25


def ring_x(k, t):
    """Block-vector entry (row k, column t): q / 8 with q in -8..8."""
    return ((5 * k + 3 * t) % 17 - 8) * 0.125


def ring_y(k, t):
    """Second block-vector entry (row k, column t): r / 16 with r in -6..6."""
    return ((3 * k + 7 * t) % 13 - 6) * 0.0625


def ring_csr(n: int, variant: int = 0) -> CSR:
    """The ring matrix of order n on the host (for sizes the host can hold)."""
    offs = ring_offsets(n)
    rows = np.arange(n, dtype=np.int64)
    lens = ring_length(rows)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=rowptr[1:])
    ie = np.repeat(rows, lens)
    je = np.arange(int(rowptr[-1]), dtype=np.int64) - np.repeat(rowptr[:-1], lens)
    return CSR(n, n, rowptr, ring_col(ie, je, offs, n).astype(np.int32), ring_val(ie, je, variant),
               f"ring_{n}")


def ring_csr_torch(n: int, device, variant: int = 0, chunk_rows: int = 1 << 22, values_only: bool = False):
    """The ring matrix of order n as torch tensors on a device (rowptr int64, col int32, val
    float64), made in row chunks to bound the temporaries. values_only: val alone (col None)."""
    import torch

    offs = torch.from_numpy(ring_offsets(n)).to(device)
    lens = ring_length(torch.arange(n, dtype=torch.int64, device=device))
    rowptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    torch.cumsum(lens, 0, out=rowptr[1:])
    nnz = int(rowptr[-1])
    col = None if values_only else torch.empty(nnz, dtype=torch.int32, device=device)
    val = torch.empty(nnz, dtype=torch.float64, device=device)
    for r0 in range(0, n, chunk_rows):
        r1 = min(n, r0 + chunk_rows)
        rows = torch.arange(r0, r1, dtype=torch.int64, device=device)
        ln = lens[r0:r1]
        p0, p1 = int(rowptr[r0]), int(rowptr[r1])
        ie = torch.repeat_interleave(rows, ln)
        je = torch.arange(p0, p1, dtype=torch.int64, device=device) - torch.repeat_interleave(rowptr[r0:r1], ln)
        if col is not None:
            col[p0:p1] = ring_col(ie, je, offs, n).to(torch.int32)
        val[p0:p1] = ring_val(ie, je, variant)
        del ie, je, rows
    return rowptr, col, val
