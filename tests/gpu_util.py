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


def colwise_relerr(got, ref, scale=None):
    """max over columns of ||got - ref|| / ||ref|| (||scale|| when given: the cancellation-safe
    denominator sum |alpha| (|A||x| + |gamma||x|) + |beta||y|)."""
    got = np.atleast_2d(got.reshape(ref.shape[0], -1))
    ref = np.atleast_2d(ref.reshape(ref.shape[0], -1))
    num = np.linalg.norm(got - ref, axis=0)
    den = np.linalg.norm(ref if scale is None else scale.reshape(ref.shape), axis=0)
    den = np.where(den == 0, 1.0, den)
    return float(np.max(num / den)) if num.size else 0.0


def abs_product(A, X):
    """|A| |X| row by row (the scale of the rounding error of A X)."""
    from synth import CSR

    Aa = CSR(A.nrows, A.ncols, A.rowptr, A.col, np.abs(A.val), A.name)
    return oracle.spmmv(Aa, np.abs(X))
