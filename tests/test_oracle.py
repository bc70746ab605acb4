"""Pins for the CPU oracle: checks against facts fixed by the paper or by mathematics,
never against the oracle itself (dense brute force, closed-form spectra, exact integer
arithmetic, correctly rounded sums, hand-derived SELL padding counts)."""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _scipy(A):
    return sp.csr_matrix((A.val, A.col, A.rowptr), shape=(A.nrows, A.ncols))


def _mats():
    return [
        synth.random_sparse(37, 37, 0.15, 3),
        synth.random_sparse(50, 29, 0.2, 4, empty_rows=5),
        synth.random_sparse(64, 64, 0.05, 5, long_row=64, empty_rows=3),
        synth.random_sparse(40, 40, 0.2, 6, duplicates=True),
        synth.laplacian2d(7),
        synth.anderson3d(4),
    ]


# ---------------------------------------------------------------- plain product


@pytest.mark.parametrize("b", [1, 3, 8])
def test_spmmv_matches_dense_brute_force(orc, b):
    for A in _mats():
        X = synth.block_vector(A.ncols, b, 11)
        Y = orc.spmmv(A, X)
        ref = A.dense() @ X
        scale = np.abs(A.dense()) @ np.abs(X)
        assert np.all(np.abs(Y - ref) <= 1e-14 * scale + 1e-300), A


def test_spmmv_matches_scipy(orc):
    A = synth.irregular(3000, band=50, seed=9)
    X = synth.block_vector(A.ncols, 4, 12)
    ref = _scipy(A) @ X
    Y = orc.spmmv(A, X)
    assert np.max(np.abs(Y - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_spmmv_integer_inputs_bit_exact(orc):
    # integer-valued A and X: every partial sum is an integer far below 2^53, so the
    # product is exact in any order and must equal the dense brute force bit for bit
    for A in _mats()[:4]:
        Ai = synth.CSR(A.nrows, A.ncols, A.rowptr, A.col, np.rint(4 * A.val), A.name)
        X = synth.int_block_vector(A.ncols, 5, 13)
        assert np.array_equal(orc.spmmv(Ai, X), Ai.dense() @ X)


def test_row_sums_and_empty_rows(orc):
    A = synth.random_sparse(60, 45, 0.2, 14, empty_rows=6, int_values=True)
    y = orc.spmmv(A, np.ones(A.ncols))
    sums = np.array([A.val[A.rowptr[i]:A.rowptr[i + 1]].sum() for i in range(A.nrows)])
    assert np.array_equal(y, sums)
    empty = A.row_lengths() == 0
    assert empty.any() and np.all(y[empty] == 0.0)


def test_laplacian_row_sums_closed_form(orc):
    # 4 - (#neighbours inside the grid) = number of missing neighbours
    N = 9
    A = synth.laplacian2d(N)
    y = orc.spmmv(A, np.ones(A.ncols)).reshape(N, N)
    xs = np.arange(N)
    missing = (xs[None, :] == 0).astype(int) + (xs[None, :] == N - 1) + (xs[:, None] == 0) + (xs[:, None] == N - 1)
    assert np.array_equal(y, missing.astype(float))


def test_dirichlet_laplacian_eigenvectors(orc):
    N = 64
    A = synth.laplacian2d(N)
    xs = np.arange(N)
    for k, l in [(1, 1), (3, 7), (64, 1), (40, 33)]:
        v = np.outer(np.sin(math.pi * l * (xs + 1) / (N + 1)), np.sin(math.pi * k * (xs + 1) / (N + 1))).ravel()
        lam = 4 - 2 * math.cos(math.pi * k / (N + 1)) - 2 * math.cos(math.pi * l / (N + 1))
        r = orc.spmmv(A, v) - lam * v
        assert np.linalg.norm(r) <= 1e-14 * np.linalg.norm(v) * 8


def test_anderson_plane_waves_without_disorder(orc):
    L = 8
    A = synth.anderson3d(L, W=0.0)
    r = np.arange(L ** 3)
    x, y, z = r % L, (r // L) % L, r // (L * L)
    for k in [(0, 0, 0), (1, 2, 3), (4, 0, 7)]:
        v = np.cos(2 * math.pi * (k[0] * x + k[1] * y + k[2] * z) / L)
        lam = -2 * sum(math.cos(2 * math.pi * kd / L) for kd in k)
        assert np.linalg.norm(orc.spmmv(A, v) - lam * v) <= 1e-13 * np.linalg.norm(v)


def test_symmetry_adjoint(orc):
    A = synth.anderson3d(6)
    x = synth.block_vector(A.nrows, 1, 1)[:, 0]
    y = synth.block_vector(A.nrows, 1, 2)[:, 0]
    lhs = np.dot(orc.spmmv(A, x), y)
    rhs = np.dot(x, orc.spmmv(A, y))
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(A.dense()) @ np.abs(x)) @ np.abs(y)


# ---------------------------------------------------------------- augmented product


def _int_case(seed=20, n=45, b=3):
    A = synth.random_sparse(n, n, 0.15, seed, int_values=True, empty_rows=2)
    X = synth.int_block_vector(n, b, seed + 1)
    Y = synth.int_block_vector(n, b, seed + 2)
    Z = synth.int_block_vector(n, b, seed + 3)
    return A, X, Y, Z


def test_aug_flag_free_is_plain_product(orc):
    A, X, Y, Z = _int_case()
    Yn, Zn, d = orc.spmmv_aug(A, X, Y=Y)
    assert np.array_equal(Yn, A.dense() @ X) and Zn is None and d is None


@pytest.mark.parametrize("flags", range(0, 256, 1))
def test_aug_every_flag_combination_exact_on_integers(orc, flags):
    # Sec. 5.3: y = alpha (A - gamma I) x + beta y, dots <y,y>, <x,y>, <x,x>, z = delta z + eta y,
    # each augmentation switched on separately. Integer data and power-of-two scalars keep
    # every operation exact, so the dense restatement must agree bit for bit.
    A, X, Y, Z = _int_case(seed=30 + flags % 7)
    b = X.shape[1]
    alpha, beta, gamma, delta, eta = 0.5, -2.0, 3.0, 0.25, -4.0
    gv = np.array([1.0, -2.0, 0.5][:b])
    Yn, Zn, d = orc.spmmv_aug(A, X, Y=Y, Z=Z, flags=flags, alpha=alpha, beta=beta, gamma=gamma,
                              gamma_v=gv, delta=delta, eta=eta)
    D = A.dense()
    g = gv[None, :] if flags & orc.VSHIFT else (gamma if flags & orc.SHIFT else 0.0)
    a = alpha if flags & orc.SCALE else 1.0
    bt = beta if flags & orc.AXPBY else 0.0
    ref = a * (D @ X - g * X) + bt * Y
    assert np.array_equal(Yn, ref)
    if flags & orc.CHAIN:
        assert np.array_equal(Zn, delta * Z + eta * ref)
    if flags & (orc.DOT_YY | orc.DOT_XY | orc.DOT_XX):
        for j in range(b):
            if flags & orc.DOT_YY:
                assert d[j] == np.dot(ref[:, j], ref[:, j])
            if flags & orc.DOT_XY:
                assert d[b + j] == np.dot(X[:, j], ref[:, j])
            if flags & orc.DOT_XX:
                assert d[2 * b + j] == np.dot(X[:, j], X[:, j])


def test_aug_beta_zero_does_not_read_y_and_delta_zero_does_not_read_z(orc):
    A, X, Y, Z = _int_case()
    Yn, Zn, _ = orc.spmmv_aug(A, X, Y=np.full_like(Y, np.nan), Z=np.full_like(Z, np.inf),
                              flags=orc.AXPBY | orc.CHAIN, beta=0.0, delta=0.0, eta=2.0)
    assert np.all(np.isfinite(Yn)) and np.all(np.isfinite(Zn))
    assert np.array_equal(Zn, 2.0 * Yn)


def test_paper_listing_sequence(orc):
    # The usage example of Sec. 5.3: first y = (A - gamma_j I) x with one shift per vector,
    # then y = (A - gamma_j I) x - 2 y chained with <x, y>.
    A, X, Y, _ = _int_case(seed=41, b=4)
    shift = np.array([1.0, 2.0, -1.0, 0.0])
    y1, _, _ = orc.spmmv_aug(A, X, flags=orc.VSHIFT, gamma_v=shift)
    y2, _, d = orc.spmmv_aug(A, X, Y=y1, flags=orc.VSHIFT | orc.AXPBY | orc.DOT_XY, beta=-2.0, gamma_v=shift)
    D = A.dense()
    r1 = D @ X - shift * X
    r2 = D @ X - shift * X - 2 * r1
    assert np.array_equal(y1, r1) and np.array_equal(y2, r2)
    assert np.array_equal(d[4:8], np.einsum("ij,ij->j", X, r2))
    assert np.all(np.isnan(d[:4])) and np.all(np.isnan(d[8:]))


def test_dot_against_correctly_rounded_sum(orc):
    a = synth.normal(51, 200001) * np.exp(synth.uniform(52, 200001, -20, 20))
    b = synth.normal(53, 200001)
    exact = math.fsum(float(u) * float(v) for u, v in zip(a.tolist(), b.tolist()))
    # products are rounded (error <= u |a_i b_i| each); the compensated sum adds about
    # 2u |exact| + O(n u^2) sum |a_i b_i|
    bound = 2.3e-16 * abs(exact) + 1.2e-16 * np.sum(np.abs(a * b)) * 1.0001
    assert abs(orc.dot(a, b) - exact) <= bound
    ai = np.arange(1, 1001, dtype=float)
    assert orc.dot(ai, ai) == 1000 * 1001 * 2001 / 6


def test_dot_compensation_beats_naive(orc):
    # 1 + many tiny terms: naive left-to-right summation loses them all
    a = np.concatenate([[1.0], np.full(100000, 1e-17)])
    assert abs(orc.dot(a, np.ones_like(a)) - (1.0 + 1e-12)) < 1e-16
    assert float(np.cumsum(a)[-1]) == 1.0


# ---------------------------------------------------------------- transpose


def test_transpose_matches_dense_and_adjoint(orc):
    for A in _mats():
        X = synth.block_vector(A.nrows, 3, 61)
        Y = orc.spmmv_T(A, X)
        ref = A.dense().T @ X
        assert np.allclose(Y, ref, rtol=0, atol=1e-13 * max(1.0, np.abs(ref).max()))
        u = synth.block_vector(A.ncols, 1, 62)[:, 0]
        v = X[:, 0]
        assert abs(np.dot(orc.spmmv_T(A, v), u) - np.dot(v, orc.spmmv(A, u))) < 1e-12 * A.nnz


def test_transpose_of_symmetric_equals_product(orc):
    A = synth.laplacian3d(5)
    X = synth.int_block_vector(A.nrows, 2, 63)
    assert np.array_equal(orc.spmmv_T(A, X), orc.spmmv(A, X))


# ---------------------------------------------------------------- SELL layout (integer work)


def test_sell_padding_matches_hand_counts(orc):
    g = json.load(open(os.path.join(GOLDEN, "sell_padding_lap2d_64.json")))
    A = synth.laplacian2d(64)
    assert A.nnz == g["nnz"]
    for case in g["cases"]:
        perm, cl, cs = orc.sell_layout(A, case["C"], case["sigma"])
        assert int(cs[-1]) == case["stored"], case


@pytest.mark.parametrize("C,sigma", [(1, 1), (4, 1), (4, 8), (32, 1), (32, 32), (32, 256), (64, 1000), (7, 5)])
def test_sell_layout_invariants(orc, C, sigma):
    A = synth.irregular(1000, band=40, max_len=300, seed=70)
    lens = A.row_lengths()
    perm, cl, cs = orc.sell_layout(A, C, sigma)
    n = A.nrows
    real = perm[:n]
    assert np.array_equal(np.sort(real), np.arange(n)) and np.all(perm[n:] == -1)
    for w in range(0, n, sigma):
        win = real[w:w + sigma]
        assert np.all((win >= w) & (win < w + sigma))  # rows stay in their window
        wl = lens[win]
        assert np.all(wl[:-1] >= wl[1:])  # descending
        eq = wl[:-1] == wl[1:]
        assert np.all(win[:-1][eq] < win[1:][eq])  # ties keep order
    slot_len = np.zeros(perm.size, dtype=np.int64)
    slot_len[:n] = lens[real]
    assert np.array_equal(cl, slot_len.reshape(-1, C).max(axis=1))
    assert np.array_equal(cs, np.concatenate([[0], np.cumsum(C * cl.astype(np.int64))]))
    if sigma % C == 0 or sigma == 1:
        _, cl1, cs1 = orc.sell_layout(A, C, 1)
        if sigma == C:
            assert cs1[-1] == cs[-1]  # sorting inside a chunk never changes its padding


def test_sell_special_cases(orc):
    A = synth.random_sparse(53, 41, 0.2, 71, empty_rows=4)
    # SELL-1-1 is CRS: identity permutation, chunk lengths = row lengths, same arrays
    perm, cl, cs = orc.sell_layout(A, 1, 1)
    assert np.array_equal(perm, np.arange(A.nrows)) and np.array_equal(cs, A.rowptr)
    scol, sval = orc.sell_fill(A, 1, perm, cl, cs)
    assert np.array_equal(scol, A.col) and np.array_equal(sval, A.val)
    # SELL-n-1 is ELLPACK: one chunk padded to the longest row, stored column-major
    n = A.nrows
    perm, cl, cs = orc.sell_layout(A, n, 1)
    m = A.row_lengths().max()
    assert cl.tolist() == [m] and cs[-1] == n * m
    scol, sval = orc.sell_fill(A, n, perm, cl, cs)
    ell_col = np.full((m, n), -1, dtype=np.int32)
    ell_val = np.zeros((m, n))
    for i in range(n):
        r = slice(A.rowptr[i], A.rowptr[i + 1])
        ell_col[: A.rowptr[i + 1] - A.rowptr[i], i] = A.col[r]
        ell_val[: A.rowptr[i + 1] - A.rowptr[i], i] = A.val[r]
    assert np.array_equal(scol, ell_col.ravel()) and np.array_equal(sval, ell_val.ravel())
    # SELL-C-1 is sliced ELLPACK: no reordering at all
    perm, cl, cs = orc.sell_layout(A, 8, 1)
    assert np.array_equal(perm[:n], np.arange(n))


def test_sell_anderson_has_no_padding(orc):
    A = synth.anderson3d(8)
    for C, sigma in [(32, 1), (64, 1), (32, 512), (128, 512)]:
        _, _, cs = orc.sell_layout(A, C, sigma)
        assert cs[-1] == A.nnz


def test_sell_fill_is_a_relayout(orc):
    # every CSR entry appears exactly once in SELL order, the rest is padding (0, -1)
    A = synth.random_sparse(70, 70, 0.1, 72, duplicates=True, empty_rows=3)
    for C, sigma in [(8, 16), (32, 70), (3, 1)]:
        perm, cl, cs = orc.sell_layout(A, C, sigma)
        scol, sval = orc.sell_fill(A, C, perm, cl, cs)
        pad = scol == -1
        assert np.all(sval[pad] == 0.0) and (~pad).sum() == A.nnz
        assert sorted(zip(scol[~pad].tolist(), sval[~pad].tolist())) == sorted(zip(A.col.tolist(), A.val.tolist()))


# ---------------------------------------------------------------- low-precision rounding


def _bf16_by_bits(x32: np.ndarray) -> np.ndarray:
    """bfloat16 rounding of float32 inputs by integer arithmetic on the bit pattern."""
    u = x32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def test_round_bf16_against_bit_arithmetic_on_float32_inputs(orc):
    x = (synth.normal(80, 100000) * np.exp(synth.uniform(81, 100000, -30, 30))).astype(np.float32)
    x = np.concatenate([x, np.float32([1.0, -1.0, 0.0, 3.0e38, 1e-40, -2.5e-39])])
    assert np.array_equal(orc.round_bf16(x.astype(np.float64)), _bf16_by_bits(x))


def test_round_bf16_ties_and_no_double_rounding(orc):
    e = 2.0 ** -8
    cases = {
        1.0 + e: 1.0,                      # tie -> even (1.0)
        1.0 + 3 * e: 1.0 + 4 * e,          # tie -> even (1 + 2^-6)
        1.0 + e + 2.0 ** -40: 1.0 + 2 * e,  # just above the tie: up (rounding via f32 would tie to 1.0)
        -(1.0 + e + 2.0 ** -40): -(1.0 + 2 * e),
        4.0: 4.0, 6.0: 6.0, -1.0: -1.0,
        3.5e38: math.inf,
    }
    got = orc.round_bf16(np.array(list(cases.keys())))
    assert got.tolist() == list(cases.values())


def test_round_f32_matches_ieee_cast(orc):
    x = synth.normal(82, 100000) * np.exp(synth.uniform(83, 100000, -80, 80))
    x = np.concatenate([x, [1 + 2.0 ** -24, 1 + 3 * 2.0 ** -24, 1e-46, 4e38]])
    with np.errstate(over="ignore"):
        ref = x.astype(np.float32).astype(np.float64)
    assert np.array_equal(orc.round_f32(x), ref)


# ---------------------------------------------------------------- CG and Chebyshev


def test_cg_manufactured_solution(orc):
    A = synth.laplacian3d(12)
    xs = synth.block_vector(A.nrows, 1, 90)[:, 0]
    b = A.dense() @ xs
    x, it = orc.cg(A, b, tol=1e-10)
    assert np.linalg.norm(b - A.dense() @ x) <= 1.05e-10 * np.linalg.norm(b)
    # eigenvalues of the 3D Dirichlet Laplacian: 6 - 2 sum cos(pi k_d / (e + 1))
    lmin = 6 - 6 * math.cos(math.pi / 13)
    assert np.linalg.norm(x - xs) <= 1.05e-10 * np.linalg.norm(b) / lmin
    assert 10 < it < A.nrows


def test_cg_refine_reduces_to_plain_cg(orc):
    """With a double inner solve on the unrounded values, an inner tolerance equal to the outer
    one and one refinement from x = 0, the refinement is plain CG: r = b - A 0 = b exactly, so
    it takes the same steps and returns the same x bit for bit."""
    A = synth.laplacian3d(11)
    b = synth.block_vector(A.nrows, 1, 93)[:, 0]
    x, it = orc.cg(A, b, tol=1e-9)
    x2, outer, inner, _ = orc.cg_refine(A, b, single=False, tol=1e-9, inner_rtol=1e-9, maxouter=1)
    assert outer == 1 and inner == it and np.array_equal(x2, x)


@pytest.mark.parametrize("vdt", ["f32", "bf16"])
def test_cg_refine_manufactured_solution(orc, vdt):
    """A float inner solve alone stalls near its unit roundoff (about 1e-7 relative); the FP64
    residual of each refinement restores the digits, so b - A x reaches 1e-10 after about
    log(1e-10) / log(inner_rtol) refinements, and x approaches x* within ||r|| / lambda_min.
    The 3D Laplacian's 6 / -1 are exact in both storage types."""
    A = synth.laplacian3d(12)
    xs = synth.block_vector(A.nrows, 1, 94)[:, 0]
    b = A.dense() @ xs
    low = orc.round_f32(A.val) if vdt == "f32" else orc.round_bf16(A.val)
    assert np.array_equal(low, A.val)
    x, outer, inner, rr = orc.cg_refine(A, b, val_low=low, tol=1e-10, inner_rtol=1e-4)
    res = np.linalg.norm(b - A.dense() @ x) / np.linalg.norm(b)
    assert res <= 1e-10 and abs(res - rr) <= 1e-3 * rr
    assert 3 <= outer <= 4  # three decades of 1e-4 reach 1e-10 (one more if a float solve falls short)
    lmin = 6 - 6 * math.cos(math.pi / 13)
    assert np.linalg.norm(x - xs) <= 1.05e-10 * np.linalg.norm(b) / lmin
    # without refinement the float solve cannot get there
    _, _, _, rr1 = orc.cg_refine(A, b, val_low=low, tol=1e-10, inner_rtol=1e-12, maxouter=1, inner_maxit=2000)
    assert rr1 > 1e-9
    # and with a perturbed inner matrix (a dropped term) refinement still converges, but slower
    bad = low.copy()
    bad[::7] *= 0.9
    _, outer2, _, rr2 = orc.cg_refine(A, b, val_low=bad, tol=1e-10, inner_rtol=1e-4)
    assert rr2 <= 1e-10 and outer2 > outer


def test_chebyshev_diagonal_closed_form(orc):
    d = synth.uniform(91, 300, -0.99, 0.99)
    n = d.size
    A = synth.CSR(n, n, np.arange(n + 1), np.arange(n, dtype=np.int32), d, "diag")
    x = synth.block_vector(n, 1, 92)[:, 0]
    mu, v = orc.chebyshev(A, x, 50, 1.0)
    m = np.arange(51)
    T = np.cos(m[:, None] * np.arccos(d)[None, :])
    assert np.allclose(mu, T @ (x * x), rtol=0, atol=1e-12 * np.dot(x, x))
    assert np.allclose(v, T[50] * x, rtol=0, atol=1e-12)


def test_chebyshev_via_eigendecomposition(orc):
    A = synth.anderson3d(5)
    s, c = 14.25 / 0.99, 0.3
    x = synth.block_vector(A.nrows, 1, 93)[:, 0]
    mu, _ = orc.chebyshev(A, x, 40, s, c)
    lam, Q = np.linalg.eigh(A.dense())
    w = (Q.T @ x) ** 2
    t = (lam - c) / s
    assert np.all(np.abs(t) < 1)
    ref = np.cos(np.arange(41)[:, None] * np.arccos(t)[None, :]) @ w
    assert np.allclose(mu, ref, rtol=0, atol=1e-11 * np.dot(x, x))


# ---------------------------------------------------------------- Chebyshev gradient


def _loss_half_sq(Y):
    return 0.5 * float(np.sum(Y * Y))


def test_cheb_apply_matches_moment_recurrence(orc):
    A = synth.anderson3d(4)
    s = 14.25 / 0.99
    x = synth.block_vector(A.nrows, 1, 94)
    for N in (1, 2, 7):
        Y = orc.cheb_apply(A, x, N, s, 0.2)
        _, vN = orc.chebyshev(A, x[:, 0], N, s, 0.2)
        assert np.allclose(Y[:, 0], vN, rtol=0, atol=1e-14 * np.abs(x).sum())


@pytest.mark.parametrize("N", [1, 2, 5])
def test_cheb_grad_against_central_differences(orc, N):
    A0 = synth.random_sparse(30, 30, 0.15, 95)
    # symmetric-pattern matrix is not required for the gradient; keep A general
    A = synth.CSR(30, 30, A0.rowptr, A0.col, A0.val, "g")
    s, c = 3.0, 0.1
    X = synth.block_vector(30, 2, 96)
    W = synth.block_vector(30, 2, 97)  # L = <W, Y>  ->  G = W
    dX, dval = orc.cheb_grad(A, X, N, s, c, W)
    h = 1e-6
    for p in range(0, A.nnz, max(1, A.nnz // 25)):
        vp, vm = A.val.copy(), A.val.copy()
        vp[p] += h
        vm[p] -= h
        Lp = np.sum(W * orc.cheb_apply(synth.CSR(30, 30, A.rowptr, A.col, vp), X, N, s, c))
        Lm = np.sum(W * orc.cheb_apply(synth.CSR(30, 30, A.rowptr, A.col, vm), X, N, s, c))
        fd = (Lp - Lm) / (2 * h)
        assert abs(dval[p] - fd) <= 1e-6 * max(1.0, abs(fd)), p
    # L is linear in X: dL/dX is exactly T_N(A~)^T W
    for i, j in [(0, 0), (7, 1), (29, 0)]:
        Xp = X.copy()
        Xp[i, j] += 1.0
        fd = np.sum(W * orc.cheb_apply(A, Xp, N, s, c)) - np.sum(W * orc.cheb_apply(A, X, N, s, c))
        assert abs(dX[i, j] - fd) <= 1e-10 * max(1.0, abs(fd))


def test_cheb_grad_symmetric_x_gradient_identity(orc):
    # A~ symmetric and L = |Y|^2 / 2: dL/dX = T_N(A~)^T Y = T_N(A~) T_N(A~) X
    A = synth.anderson3d(5)
    s, N = 14.25 / 0.99, 12
    X = synth.block_vector(A.nrows, 3, 98)
    Y = orc.cheb_apply(A, X, N, s)
    dX, _ = orc.cheb_grad(A, X, N, s, 0.0, Y)
    ref = orc.cheb_apply(A, Y, N, s)
    assert np.allclose(dX, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_cheb_grad_diagonal_closed_form(orc):
    # A = diag(d): Y_i = T_N(d_i / s) X_i, dL/dd_i = G_i X_i T_N'(d_i / s) / s with
    # T_N'(cos t) = N sin(N t) / sin(t)
    n, N, s = 50, 9, 1.5
    d = synth.uniform(99, n, -1.2, 1.2)
    A = synth.CSR(n, n, np.arange(n + 1), np.arange(n, dtype=np.int32), d, "diag")
    X = synth.block_vector(n, 1, 100)
    G = synth.block_vector(n, 1, 101)
    _, dval = orc.cheb_grad(A, X, N, s, 0.0, G)
    t = np.arccos(d / s)
    dT = N * np.sin(N * t) / np.sin(t)
    assert np.allclose(dval, G[:, 0] * X[:, 0] * dT / s, rtol=1e-11, atol=1e-13)


def test_pattern_outer_is_gradient_of_bilinear_form(orc):
    A = synth.random_sparse(40, 25, 0.2, 102, duplicates=True)
    G = synth.block_vector(40, 3, 103)
    X = synth.block_vector(25, 3, 104)
    dval = orc.pattern_outer(A, G, X)
    rows = np.repeat(np.arange(40), A.row_lengths())
    assert np.allclose(dval, np.einsum("pj,pj->p", G[rows], X[A.col]), rtol=1e-15, atol=1e-15)


# ---------------------------------------------------------------- tall-skinny kernels


def test_tsm_kernels_against_dense(orc):
    V = synth.block_vector(500, 5, 150)
    W = synth.block_vector(500, 3, 151)
    X0 = synth.block_vector(5, 3, 152)
    assert np.allclose(orc.tsmttsm(V, W, 2.0, -1.0, X0), 2.0 * V.T @ W - X0, rtol=0, atol=1e-12)
    assert np.allclose(orc.tsmm(V, X0, 0.5, 2.0, W), 0.5 * V @ X0 + 2.0 * W, rtol=0, atol=1e-13)
    S = synth.block_vector(5, 5, 153)
    assert np.allclose(orc.tsmm_inplace(V, S, 1.5, -0.5), 1.5 * V @ S - 0.5 * V, rtol=0, atol=1e-13)
    # integer data: exact in any order
    Vi, Wi = synth.int_block_vector(300, 4, 154), synth.int_block_vector(300, 2, 155)
    assert np.array_equal(orc.tsmttsm(Vi, Wi), Vi.T @ Wi)
    assert np.array_equal(orc.tsmttsm(Vi, Wi, kahan=True), Vi.T @ Wi)


def test_tsmttsm_kahan_is_accurate(orc):
    # ill-conditioned inner products: the compensated sum stays within a few ulps of the
    # correctly rounded result, the plain sum does not
    n = 100000
    a = synth.normal(156, n) * np.exp(synth.uniform(157, n, -15, 15))
    V = np.stack([a, np.ones(n)], axis=1)
    W = np.stack([synth.normal(158, n), -np.ones(n) * 1e-3], axis=1)
    exact = [[math.fsum((V[:, l] * W[:, j]).tolist()) for j in range(2)] for l in range(2)]
    Xk = orc.tsmttsm(V, W, kahan=True)
    for l in range(2):
        for j in range(2):
            bound = 4.5e-16 * abs(exact[l][j]) + 1.2e-16 * float(np.sum(np.abs(V[:, l] * W[:, j])))
            assert abs(Xk[l, j] - exact[l][j]) <= bound


def test_cheb_filter_is_matrix_exponential(orc):
    """exp(t x) = I_0(t) + 2 sum_m I_m(t) T_m(x) (the Chebyshev expansion of the exponential);
    with 41 terms at t = 1.7 the truncation is far below rounding, so the filter with these
    coefficients equals the dense matrix exponential of A~ applied to X."""
    import scipy.linalg
    import scipy.special

    A = synth.anderson3d(5, W=4.0)
    s = (6 + 2.0) / 0.9
    D = sp.csr_matrix((A.val, A.col, A.rowptr), shape=(A.nrows, A.ncols)).toarray()
    X = synth.block_vector(A.nrows, 3, 5)
    t, N = 1.7, 40
    coef = np.array([scipy.special.iv(m, t) * (1.0 if m == 0 else 2.0) for m in range(N + 1)])
    for c in (0.0, 0.4):
        Z = orc.cheb_filter(A, X, coef, s, c)
        ref = scipy.linalg.expm(t * (D - c * np.eye(A.nrows)) / s) @ X
        assert np.abs(Z - ref).max() <= 1e-14 * np.abs(ref).max()


def test_cheb_filter_diagonal_closed_form_and_degenerate_cases(orc):
    rng = np.random.default_rng(8)
    n = 50
    d = rng.uniform(-3, 3, n)
    A = synth.CSR(n, n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), d, "diag")
    s, c = 3.5, 0.25
    X = synth.block_vector(n, 2, 9)
    coef = rng.normal(size=31)
    th = np.arccos((d - c) / s)
    ref = (np.cos(np.outer(th, np.arange(31))) @ coef)[:, None] * X
    assert np.abs(orc.cheb_filter(A, X, coef, s, c) - ref).max() <= 1e-13 * np.abs(ref).max()
    # degree 0 is the scaled input; a unit coefficient vector picks one Chebyshev term
    assert np.array_equal(orc.cheb_filter(A, X, [2.5], s, c), 2.5 * X)
    e = np.zeros(8)
    e[7] = 1.0
    assert np.abs(orc.cheb_filter(A, X, e, s, c) - orc.cheb_apply(A, X, 7, s, c)).max() <= 1e-14


def test_oracle_triad_and_threads(orc):
    """The host bandwidth probe computes a = b + s c exactly (one rounding per element), and
    the thread setting takes effect and can be restored."""
    n = 100_003
    b = synth.uniform(synth.SEED_X, n, -1.0, 1.0)
    c = synth.uniform(synth.SEED_Y, n, -1.0, 1.0)
    a = np.zeros(n)
    orc.triad(a, b, c, 0.75)
    assert np.array_equal(a, b + 0.75 * c)  # numpy rounds s*c, then the sum: the same two steps
    before = orc.num_threads()
    orc.set_num_threads(1)
    assert orc.num_threads() == 1
    orc.set_num_threads(before)
    assert orc.num_threads() == before
    orc.set_num_threads(0)  # ignored
    assert orc.num_threads() == before


def test_oracle_fma_build_contracts(orc):
    """The two oracle builds differ exactly where contraction must change the bits: the row
    [1, a] times [c, x] with a = x = 1 + 2^-30 and c = -(1 + 2^-29). Without FMA, a x rounds to
    1 + 2^-29 and the sum is 0; with FMA, the sum is the exact 2^-60."""
    a = 1.0 + 2.0 ** -30
    A = synth.CSR(1, 2, np.array([0, 2], np.int64), np.array([0, 1], np.int32), np.array([1.0, a]), "fma_pin")
    X = np.array([-(1.0 + 2.0 ** -29), a])
    assert orc.spmmv(A, X)[0] == 0.0
    assert orc.spmmv(A, X, fma=True)[0] == 2.0 ** -60
    # and on ordinary data both builds agree to rounding
    B = synth.anderson3d(8)
    x = synth.block_vector(B.nrows, 1, synth.SEED_X)[:, 0]
    y0, y1 = orc.spmmv(B, x), orc.spmmv(B, x, fma=True)
    assert np.max(np.abs(y0 - y1)) <= 1e-14 * np.max(np.abs(y0))
