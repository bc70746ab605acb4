"""Helpers shared by the GPU tests: device placement, flag mapping, error metrics."""
import numpy as np

import oracle
import paper_1507_08101_amd as sc

FLAG_PAIRS = [(sc.SHIFT, oracle.SHIFT), (sc.VSHIFT, oracle.VSHIFT), (sc.SCALE, oracle.SCALE),
              (sc.AXPBY, oracle.AXPBY), (sc.DOT_YY, oracle.DOT_YY), (sc.DOT_XY, oracle.DOT_XY),
              (sc.DOT_XX, oracle.DOT_XX), (sc.CHAIN, oracle.CHAIN)]


def to_oracle_flags(f: int) -> int:
    return sum(o for l, o in FLAG_PAIRS if f & l)


def dev(a, dtype=None):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def host(t):
    import torch

    torch.cuda.synchronize()
    return t.detach().to("cpu").double().numpy()


# A column's reference norm counts as "tiny" (cancellation) when it is below this fraction of the
# norm of the error scale |alpha|(|A||x| + |gamma||x|) + |beta||y|. Above it, the FP64 rounding error
# of a row sum (at most a few hundred ulps of the scale in these tests) divided by ||y_ref|| stays
# below 1e-12 only if the scale is within about a factor 1e3 of ||y_ref||.
TINY = 1e-3
# columns checked by colwise_relerr, and how many of them divided by the error scale
RELERR_STATS = {"columns": 0, "scale_denominator": 0}


def colwise_relerr(got, ref, scale=None):
    """Max over columns of the normwise relative error ||got - ref||_2 / ||ref||_2.

    Only a column whose ||ref|| is tiny (below TINY * ||scale||, cancellation) divides by the norm
    of the error scale instead, when one is given; a column that is exactly zero in the reference
    divides by 1."""
    got = np.atleast_2d(got.reshape(ref.shape[0], -1))
    ref = np.atleast_2d(ref.reshape(ref.shape[0], -1))
    num = np.linalg.norm(got - ref, axis=0)
    den = np.linalg.norm(ref, axis=0)
    if scale is not None:
        sden = np.linalg.norm(scale.reshape(ref.shape), axis=0)
        tiny = den < TINY * sden
        RELERR_STATS["scale_denominator"] += int(np.count_nonzero(tiny))
        den = np.where(tiny, sden, den)
    RELERR_STATS["columns"] += int(num.size)
    den = np.where(den == 0, 1.0, den)
    return float(np.max(num / den)) if num.size else 0.0


def gamma_bound(k, u=2.0 ** -53):
    """gamma_k = k u / (1 - k u): the bound on the relative error of k rounded operations
    (elementwise, k may be an array)."""
    k = np.asarray(k, dtype=np.float64)
    return k * u / (1.0 - k * u)


def abs_product(A, X):
    """|A| |X| row by row (the scale of the rounding error of A X)."""
    from synth import CSR

    Aa = CSR(A.nrows, A.ncols, A.rowptr, A.col, np.abs(A.val), A.name)
    return oracle.spmmv(Aa, np.abs(X))


def rounded_matrix(A, dt):
    """A with its values rounded to the storage type dt (RNE directly from the double)."""
    from synth import CSR

    if dt == "f64":
        return A
    val = oracle.round_f32(A.val) if dt == "f32" else oracle.round_bf16(A.val)
    return CSR(A.nrows, A.ncols, A.rowptr, A.col, val, A.name + "_" + dt)


def assert_lowprec_product(got, A, X32, dt, extra=0, what=""):
    """The FP32-accumulated product of an f32/bf16-valued matrix with FP32 vectors against the
    exact product of the rounded inputs (the oracle's FP64 product of the rounded values and
    vectors, exact to far below the FP32 bound): per element
    |got - exact| <= gamma_{k+extra}(u = 2^-24) (|A~||x|)_i with k the row length, the deterministic
    bound of a k-term sum of products in FP32 in any order, with or without fused multiply-adds."""
    Ar = rounded_matrix(A, dt)
    exact = oracle.spmmv(Ar, X32)
    k = A.row_lengths().reshape(-1, 1) + extra
    bound = gamma_bound(k, 2.0 ** -24) * abs_product(Ar, X32)
    bad = np.abs(got - exact) > bound
    assert not bad.any(), (what, int(bad.sum()), float(np.max(np.abs(got - exact) / np.where(bound > 0, bound, 1))))
    return exact
