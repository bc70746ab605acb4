"""CPU FP64 oracle for the SELL-C-sigma augmented SpMMV (GHOST paper, Sec. 5.1-5.3).

TEST INFRASTRUCTURE ONLY. This package is the independent checker: plain C routines
(``oracle.c``) on CSR input in IEEE double, wrapped here with ctypes and numpy. Only the
test suite, the smoke check and the benchmark's CPU-baseline leg may import it; the
library (``paper_1507_08101_amd``) never does, and the two share no code.

Functions take a CSR-like object with ``nrows, ncols, rowptr (int64), col (int32),
val (float64)`` and row-major float64 numpy block vectors.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

from . import build as _build

SHIFT, VSHIFT, SCALE, AXPBY, DOT_YY, DOT_XY, DOT_XX, CHAIN = (1, 2, 4, 8, 16, 32, 64, 128)

_libs = {}
_P = ct.c_void_p
_I64 = ct.c_int64
_D = ct.c_double


def lib(fma: bool = False):
    """Load (building on first use if absent) the oracle shared library; fma: the build whose
    multiply-adds are contracted into FMAs (for the rounding-noise envelope only)."""
    path = _build.LIB_FMA if fma else _build.LIB
    if path not in _libs:
        if not os.path.exists(path):
            _build.build()
        L = ct.CDLL(path)
        L.orc_spmmv.argtypes = [_I64, _P, _P, _P, _I64, _P, _I64, _P, _I64]
        L.orc_spmmv_aug.argtypes = [_I64, _I64, _P, _P, _P, _I64, _P, _I64, _P, _I64, _P, _I64,
                                    ct.c_uint, _D, _D, _D, _P, _D, _D, _P]
        L.orc_dot.argtypes = [_I64, _P, _I64, _P, _I64]
        L.orc_dot.restype = _D
        L.orc_spmmv_T.argtypes = [_I64, _I64, _P, _P, _P, _I64, _P, _I64, _P, _I64]
        L.orc_sell_layout.argtypes = [_I64, _P, _I64, _I64, _P, _P, _P]
        L.orc_sell_fill.argtypes = [_I64, _P, _P, _P, _I64, _P, _P, _P, _P, _P]
        L.orc_round_bf16.argtypes = [_I64, _P, _P]
        L.orc_round_f32.argtypes = [_I64, _P, _P]
        L.orc_cg.argtypes = [_I64, _P, _P, _P, _P, _P, _D, _I64, _P]
        L.orc_cg_refine.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _D, _D, _I64, _I64, ct.c_int, _P, _P, _P]
        L.orc_chebyshev.argtypes = [_I64, _P, _P, _P, _P, _I64, _D, _D, _P, _P]
        L.orc_num_threads.restype = ct.c_int
        L.orc_set_num_threads.argtypes = [ct.c_int]
        L.orc_set_num_threads.restype = None
        L.orc_triad.argtypes = [_I64, _P, _P, _P, _D]
        L.orc_cheb_apply.argtypes = [_I64, _P, _P, _P, _I64, _P, _I64, _D, _D, _P]
        L.orc_cheb_grad.argtypes = [_I64, _P, _P, _P, _I64, _P, _I64, _D, _D, _P, _P, _P]
        L.orc_pattern_outer.argtypes = [_I64, _P, _P, _I64, _P, _P, _P]
        L.orc_cheb_filter.argtypes = [_I64, _P, _P, _P, _I64, _P, _I64, _P, _D, _D, _P]
        L.orc_tsmttsm.argtypes = [_I64, _I64, _I64, _D, _P, _P, _D, _P, ct.c_int]
        L.orc_tsmm.argtypes = [_I64, _I64, _I64, _D, _P, _P, _D, _P]
        L.orc_tsmm_inplace.argtypes = [_I64, _I64, _D, _P, _P, _D]
        _libs[path] = L
    return _libs[path]


def _p(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (rc={rc})")


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's later parallel loops."""
    lib().orc_set_num_threads(int(n))


def triad(a, b, c, s):
    """STREAM triad a = b + s c in place on float64 arrays (host bandwidth probe)."""
    assert a.dtype == b.dtype == c.dtype == np.float64 and a.shape == b.shape == c.shape
    assert a.flags.c_contiguous and b.flags.c_contiguous and c.flags.c_contiguous
    _check(lib().orc_triad(a.size, _p(a), _p(b), _p(c), float(s)), "triad")


def spmmv(A, X, fma=False):
    """Y = A X for a row-major block vector X (ncols x b) or a vector (ncols,); fma: the
    FMA-contracted build."""
    X = _f64(X)
    vec = X.ndim == 1
    X2 = X.reshape(-1, 1) if vec else X
    b = X2.shape[1]
    Y = np.empty((A.nrows, b))
    _check(lib(fma).orc_spmmv(A.nrows, _p(A.rowptr), _p(A.col), _p(A.val), b, _p(X2), b, _p(Y), b), "spmmv")
    return Y[:, 0] if vec else Y


def spmmv_aug(A, X, Y=None, Z=None, flags=0, alpha=1.0, beta=0.0, gamma=0.0, gamma_v=None,
              delta=0.0, eta=1.0):
    """Augmented product; returns (Y_new, Z_new or None, dot[3b] or None). Inputs are not modified."""
    X = _f64(X)
    if X.ndim == 1:
        X = X.reshape(-1, 1)
    b = X.shape[1]
    Yn = np.zeros((A.nrows, b)) if Y is None else _f64(Y).reshape(A.nrows, b).copy()
    Zn = None
    if flags & CHAIN:
        Zn = np.zeros((A.nrows, b)) if Z is None else _f64(Z).reshape(A.nrows, b).copy()
    gv = None if gamma_v is None else _f64(gamma_v)
    dot = np.full(3 * b, np.nan) if flags & (DOT_YY | DOT_XY | DOT_XX) else None
    rc = lib().orc_spmmv_aug(A.nrows, A.ncols, _p(A.rowptr), _p(A.col), _p(A.val), b, _p(X), b,
                             _p(Yn), b, _p(Zn), b, flags, alpha, beta, gamma, _p(gv), delta, eta, _p(dot))
    _check(rc, "spmmv_aug")
    return Yn, Zn, dot


def dot(a, b):
    a = _f64(a)
    b = _f64(b)
    assert a.shape == b.shape and a.ndim == 1
    return lib().orc_dot(a.size, _p(a), 1, _p(b), 1)


def spmmv_T(A, X):
    X = _f64(X)
    vec = X.ndim == 1
    X2 = X.reshape(-1, 1) if vec else X
    b = X2.shape[1]
    Y = np.empty((A.ncols, b))
    _check(lib().orc_spmmv_T(A.nrows, A.ncols, _p(A.rowptr), _p(A.col), _p(A.val), b, _p(X2), b,
                             _p(Y), b), "spmmv_T")
    return Y[:, 0] if vec else Y


def sell_layout(A, C, sigma):
    """(perm int32[nch*C], cl int32[nch], cs int64[nch+1]) by brute force."""
    nch = (A.nrows + C - 1) // C
    perm = np.empty(nch * C, dtype=np.int32)
    cl = np.empty(nch, dtype=np.int32)
    cs = np.empty(nch + 1, dtype=np.int64)
    _check(lib().orc_sell_layout(A.nrows, _p(A.rowptr), C, sigma, _p(perm), _p(cl), _p(cs)), "sell_layout")
    return perm, cl, cs


def sell_fill(A, C, perm, cl, cs):
    """(scol int32[stored], sval float64[stored]) in SELL order; padding is (-1, 0.0)."""
    stored = int(cs[-1])
    scol = np.empty(stored, dtype=np.int32)
    sval = np.empty(stored, dtype=np.float64)
    _check(lib().orc_sell_fill(A.nrows, _p(A.rowptr), _p(A.col), _p(A.val), C, _p(perm), _p(cl),
                               _p(cs), _p(scol), _p(sval)), "sell_fill")
    return scol, sval


def round_bf16(a):
    a = _f64(a)
    out = np.empty_like(a)
    lib().orc_round_bf16(a.size, _p(a), _p(out))
    return out


def round_f32(a):
    a = _f64(a)
    out = np.empty_like(a)
    lib().orc_round_f32(a.size, _p(a), _p(out))
    return out


def cg(A, bvec, x0=None, tol=1e-10, maxit=100000):
    """FP64 CG; returns (x, iterations)."""
    bvec = _f64(bvec)
    x = np.zeros(A.nrows) if x0 is None else _f64(x0).copy()
    it = ct.c_int64(0)
    _check(lib().orc_cg(A.nrows, _p(A.rowptr), _p(A.col), _p(A.val), _p(bvec), _p(x), tol, maxit,
                        ct.byref(it)), "cg")
    return x, it.value


def cg_refine(A, bvec, val_low=None, x0=None, tol=1e-10, inner_rtol=1e-4, inner_maxit=100000, maxouter=1000,
              single=True):
    """Iterative refinement with an inner CG in float (single) or double on the values val_low
    (default: A's values); returns (x, outer refinements, inner iterations, final relres)."""
    bvec = _f64(bvec)
    vl = A.val if val_low is None else _f64(val_low)
    x = np.zeros(A.nrows) if x0 is None else _f64(x0).copy()
    o, i, rr = ct.c_int64(0), ct.c_int64(0), ct.c_double(0.0)
    _check(lib().orc_cg_refine(A.nrows, _p(A.rowptr), _p(A.col), _p(A.val), _p(vl), _p(bvec), _p(x), tol,
                               inner_rtol, inner_maxit, maxouter, 1 if single else 0, ct.byref(o), ct.byref(i),
                               ct.byref(rr)), "cg_refine")
    return x, o.value, i.value, rr.value


def chebyshev(A, x, M, s, c=0.0, fma=False):
    """Direct KPM moments mu[0..M] = <x, T_m(A~) x> with A~ = (A - cI)/s, and v_M; fma: the
    FMA-contracted build."""
    x = _f64(x)
    mu = np.empty(M + 1)
    v = np.empty(A.nrows)
    _check(lib(fma).orc_chebyshev(A.nrows, _p(A.rowptr), _p(A.col), _p(A.val), _p(x), M, s, c, _p(mu),
                               _p(v)), "chebyshev")
    return mu, v


def cheb_apply(A, X, N, s, c=0.0):
    """Y = T_N((A - cI)/s) X for a row-major block X (n x b)."""
    X = _f64(X)
    X2 = X.reshape(A.nrows, -1)
    b = X2.shape[1]
    Y = np.empty_like(X2)
    _check(lib().orc_cheb_apply(A.nrows, _p(A.rowptr), _p(A.col), _p(A.val), b, _p(X2), N, s, c, _p(Y)),
           "cheb_apply")
    return Y.reshape(X.shape)


def cheb_filter(A, X, coef, s, c=0.0):
    """Z = sum_m coef[m] T_m((A - cI)/s) X for a row-major block X (n x b); N = len(coef) - 1."""
    X = _f64(X)
    X2 = X.reshape(A.nrows, -1)
    b = X2.shape[1]
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    Z = np.empty_like(X2)
    _check(lib().orc_cheb_filter(A.nrows, _p(A.rowptr), _p(A.col), _p(A.val), b, _p(X2), len(coef) - 1, _p(coef),
                                 s, c, _p(Z)), "cheb_filter")
    return Z.reshape(X.shape)


def cheb_grad(A, X, N, s, c, G):
    """(dL/dX, dL/dval) for Y = T_N(A~) X and dL/dY = G, by the stored-vector adjoint recurrence."""
    X = _f64(X)
    X2 = X.reshape(A.nrows, -1)
    G2 = _f64(G).reshape(X2.shape)
    b = X2.shape[1]
    dX = np.empty_like(X2)
    dval = np.empty(A.nnz)
    _check(lib().orc_cheb_grad(A.nrows, _p(A.rowptr), _p(A.col), _p(A.val), b, _p(X2), N, s, c, _p(G2), _p(dX),
                               _p(dval)), "cheb_grad")
    return dX.reshape(X.shape), dval


def pattern_outer(A, G, X):
    """dval[p] = sum_j G[row(p), j] X[col(p), j] (CSR order)."""
    G2 = _f64(G).reshape(A.nrows, -1)
    X2 = _f64(X).reshape(A.ncols, -1)
    dval = np.empty(A.nnz)
    _check(lib().orc_pattern_outer(A.nrows, _p(A.rowptr), _p(A.col), G2.shape[1], _p(G2), _p(X2), _p(dval)),
           "pattern_outer")
    return dval


def tsmttsm(V, W, alpha=1.0, beta=0.0, X=None, kahan=False):
    """X = alpha V^T W + beta X (V: n x m, W: n x k)."""
    V, W = _f64(V), _f64(W)
    n, m = V.shape
    k = W.shape[1]
    Xo = np.zeros((m, k)) if X is None else _f64(X).copy()
    _check(lib().orc_tsmttsm(n, m, k, alpha, _p(V), _p(W), beta, _p(Xo), 1 if kahan else 0), "tsmttsm")
    return Xo


def tsmm(V, X, alpha=1.0, beta=0.0, W=None):
    """W = alpha V X + beta W (V: n x m, X: m x k)."""
    V, X = _f64(V), _f64(X)
    n, m = V.shape
    k = X.shape[1]
    Wo = np.zeros((n, k)) if W is None else _f64(W).copy()
    _check(lib().orc_tsmm(n, m, k, alpha, _p(V), _p(X), beta, _p(Wo)), "tsmm")
    return Wo


def tsmm_inplace(V, X, alpha=1.0, beta=0.0):
    """V = alpha V X + beta V (X: m x m); returns the new V."""
    Vo = _f64(V).copy()
    X = _f64(X)
    n, m = Vo.shape
    _check(lib().orc_tsmm_inplace(n, m, alpha, _p(Vo), _p(X), beta), "tsmm_inplace")
    return Vo


# ------------------------------------------------------------------ KPM density of states
# Textbook kernel polynomial method (Weisse, Wellein, Alvermann, Fehske, Rev. Mod. Phys. 78,
# 275 (2006)); the paper names KPM as a user of the augmented block product but does not
# define the reconstruction, so these follow that review.


def jackson(N):
    """Jackson damping factors g_0..g_{N-1} for N Chebyshev moments (closed form of the
    optimal positive kernel)."""
    m = np.arange(N, dtype=np.float64)
    q = np.pi / (N + 1)
    return ((N - m + 1) * np.cos(q * m) + np.sin(q * m) / np.tan(q)) / (N + 1)


def kpm_dos(mu, b, E, s, c=0.0, kernel="jackson"):
    """Density of states per unit energy at the energies E from block KPM moments.

    mu: (nmom * b) moments laid out moment-major (column j of moment m at m * b + j), as
    <v_j, T_m(A~) v_j> with A~ = (A - cI)/s. The block estimate of the normalised trace is
    sum_j mu[m, j] / sum_j mu[0, j]; it is damped (Jackson, or "none"), and the density is
    (g_0 mu_0 + 2 sum_{m>=1} g_m mu_m T_m(x)) / (pi sqrt(1 - x^2)) / s at x = (E - c)/s, with
    T_m(x) = cos(m arccos x); energies with |x| >= 1 get 0."""
    mu = np.asarray(mu, dtype=np.float64).reshape(-1, b)
    tot = mu.sum(axis=1)
    mt = tot / tot[0]
    N = mt.shape[0]
    g = jackson(N) if kernel == "jackson" else np.ones(N)
    x = (np.asarray(E, dtype=np.float64) - c) / s
    rho = np.zeros_like(x)
    inside = np.abs(x) < 1.0
    xi = x[inside]
    th = np.arccos(xi)
    m = np.arange(1, N, dtype=np.float64)
    series = g[0] * mt[0] + 2.0 * (g[1:, None] * mt[1:, None] * np.cos(m[:, None] * th[None, :])).sum(axis=0)
    rho[inside] = series / (np.pi * np.sqrt(1.0 - xi * xi)) / s
    return rho
