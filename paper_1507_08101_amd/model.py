"""Traffic and flop model of the SELL-C-sigma (augmented) SpMMV.

The product is bound by memory bandwidth (GHOST paper Sec. 4.1, 5.2): its minimum code
balance is one matrix value plus one column index per nonzero for two flops, i.e. 6 bytes
per flop for 8-byte values and 4-byte indices.

``bytes_min`` counts what the method must move at least once per call: every true
nonzero (value + 32-bit index), every input vector element once, the output written once
(read too when beta != 0), the chained vector read (delta != 0) and written, the row
permutation (when sigma sorted anything) and the chunk metadata (a 4-byte length and an
8-byte start per chunk). ``bytes_sell`` is the same with the padded entry count, i.e. what
the SELL-C-sigma layout itself streams.
"""
from __future__ import annotations


def min_code_balance(value_bytes: int, index_bytes: int = 4, flops_per_nonzero: int = 2) -> float:
    """Bytes per flop of the plain SpMV at one value + one index per nonzero."""
    return (value_bytes + index_bytes) / flops_per_nonzero


def index_width_reduction(value_bytes: int) -> float:
    """Fraction of minimum traffic saved by 32- instead of 64-bit column indices."""
    return 1.0 - (value_bytes + 4) / (value_bytes + 8)


def min_chunk_height(simd_bytes, element_bytes: int) -> int:
    """Smallest chunk height that fills the widest SIMD unit of a heterogeneous node."""
    return max(simd_bytes) // element_bytes


def flops(nnz: int, b: int) -> int:
    """Two flops per true nonzero per vector (padding is not counted)."""
    return 2 * nnz * b


def bytes_min(nnz: int, nrows: int, ncols: int, b: int, value_bytes: int, vec_bytes: int, *,
              read_y: bool = False, chain: bool = False, read_z: bool = False, has_perm: bool = False,
              nchunks: int = 0, entries: int | None = None) -> int:
    e = nnz if entries is None else entries
    matrix = e * (value_bytes + 4)
    x = ncols * b * vec_bytes
    y = nrows * b * vec_bytes * (2 if read_y else 1)
    z = nrows * b * vec_bytes * ((2 if read_z else 1) if chain else 0)
    perm = 4 * nrows if has_perm else 0
    meta = 12 * nchunks
    return matrix + x + y + z + perm + meta


def bytes_sell(stored: int, nrows: int, ncols: int, b: int, value_bytes: int, vec_bytes: int, **kw) -> int:
    return bytes_min(0, nrows, ncols, b, value_bytes, vec_bytes, entries=stored, **kw)
