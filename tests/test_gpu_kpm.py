"""GPU parity of the kernel polynomial method recurrence (sell_kpm) and of one augmented
product at the full size of the 128^3 Anderson workload."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import abs_product, colwise_relerr, dev, host

pytestmark = pytest.mark.gpu

W = 16.5


@pytest.fixture(scope="module")
def sc():
    import torch

    import paper_1507_08101_amd as sc

    assert torch.cuda.is_available()
    sc.lib()
    return sc


def _scale(W=W):
    # Gershgorin: |lambda| <= 6 + W/2, with a 1 % margin
    return (6 + W / 2) / 0.99


@pytest.mark.parametrize("b", [1, 3, 8])
def test_kpm_moments_match_direct_chebyshev(sc, b):
    import torch

    A = synth.anderson3d(10)
    M = 40
    s = _scale()
    V0 = synth.block_vector(A.nrows, b, synth.SEED_X)
    Vd = dev(V0)
    Wd = torch.zeros_like(Vd)
    mu = torch.zeros((2 * M + 1) * b, dtype=torch.float64, device="cuda:0")
    Mx = sc.SellMatrix.from_csr(A, C=32, sigma=1)
    last_in_w = sc.sell_kpm(Mx, Vd, Wd, M, s, 0.0, mu)
    mu_h = host(mu).reshape(2 * M + 1, b)
    vlast = host(Wd if last_in_w else Vd)
    for j in range(b):
        ref_mu, ref_v = oracle.chebyshev(A, V0[:, j], 2 * M, s, 0.0)
        nx = float(V0[:, j] @ V0[:, j])
        assert np.all(np.abs(mu_h[:, j] - ref_mu) <= 1e-11 * nx), j
        _, vM = oracle.chebyshev(A, V0[:, j], M, s, 0.0)
        assert np.linalg.norm(vlast[:, j] - vM) <= 1e-11 * np.linalg.norm(V0[:, j])
    Mx.close()


def test_kpm_step_local_parity(sc):
    # each step compared with the oracle applied to the same device input
    import torch

    A = synth.anderson3d(16)
    s = _scale()
    b = 2
    Mx = sc.SellMatrix.from_csr(A, C=32, sigma=1)
    x = dev(synth.block_vector(A.nrows, b, 3))
    y = dev(synth.block_vector(A.nrows, b, 4))
    dot = torch.zeros(3 * b, dtype=torch.float64, device="cuda:0")
    for step in range(20):
        xin, yin = host(x), host(y)
        sc.sell_spmmv_aug(Mx, x, y, flags=sc.SCALE | sc.SHIFT | sc.AXPBY | sc.DOT_YY | sc.DOT_XY,
                          alpha=2.0 / s, gamma=0.3, beta=-1.0, dot=dot)
        ref, _, rd = oracle.spmmv_aug(A, xin, Y=yin, flags=oracle.SCALE | oracle.SHIFT | oracle.AXPBY
                                      | oracle.DOT_YY | oracle.DOT_XY, alpha=2.0 / s, gamma=0.3, beta=-1.0)
        scale = (2.0 / s) * (abs_product(A, xin) + 0.3 * np.abs(xin)) + np.abs(yin)
        assert colwise_relerr(host(y), ref, scale) <= 1e-12, step
        d = host(dot)
        assert np.all(np.abs(d[:2 * b] - rd[:2 * b]) <= 1e-12 * np.abs(rd[:2 * b]) + 1e-300), step
        x, y = y, x


def test_chebyshev_diagonal_closed_form_on_gpu(sc):
    import torch

    n = 4000
    d = synth.uniform(5, n, -0.95, 0.95)
    A = synth.CSR(n, n, np.arange(n + 1), np.arange(n, dtype=np.int32), d, "diag")
    Mx = sc.SellMatrix.from_csr(A, C=64, sigma=1)
    x = synth.block_vector(n, 1, 6)
    M = 30
    mu = torch.zeros(2 * M + 1, dtype=torch.float64, device="cuda:0")
    V = dev(x)
    Wd = torch.zeros_like(V)
    sc.sell_kpm(Mx, V, Wd, M, 1.0, 0.0, mu)
    m = np.arange(2 * M + 1)
    ref = np.cos(m[:, None] * np.arccos(d)[None, :]) @ (x[:, 0] ** 2)
    assert np.all(np.abs(host(mu) - ref) <= 1e-11 * float(x[:, 0] @ x[:, 0]))
    Mx.close()


@pytest.mark.parametrize("b", [1, 8])
def test_full_size_anderson_128_sampled_rows(sc, b):
    """The workload the benchmark times (128^3 periodic Anderson, SELL-32-1), one KPM step,
    checked on 4096 sampled rows computed one by one, and the dots as a property of the
    whole output."""
    import torch

    A = synth.anderson3d(128)
    s = _scale()
    Mx = sc.SellMatrix.from_csr(A, C=32, sigma=1)
    X = synth.block_vector(A.nrows, b, synth.SEED_X)
    Y0 = synth.block_vector(A.nrows, b, synth.SEED_Y)
    Xd, Yd = dev(X), dev(Y0)
    dot = torch.zeros(3 * b, dtype=torch.float64, device="cuda:0")
    alpha, gamma = 2.0 / s, 0.0
    sc.sell_spmmv_aug(Mx, Xd, Yd, flags=sc.SCALE | sc.SHIFT | sc.AXPBY | sc.DOTS, alpha=alpha, gamma=gamma,
                      beta=-1.0, dot=dot)
    y = host(Yd)
    rows = np.sort(synth.randint(77, 4096, 0, A.nrows - 1))
    rows = np.unique(np.concatenate([rows, [0, A.nrows - 1]]))
    for i in rows:
        p0, p1 = A.rowptr[i], A.rowptr[i + 1]
        acc = np.zeros(b)
        for p in range(p0, p1):
            acc = acc + A.val[p] * X[A.col[p]]
        ref = alpha * (acc - gamma * X[i]) - Y0[i]
        sc_ = alpha * (np.abs(A.val[p0:p1]) @ np.abs(X[A.col[p0:p1]])) + np.abs(Y0[i])
        assert np.all(np.abs(y[i] - ref) <= 1e-12 * sc_ * 8), i
    d = host(dot)
    for j in range(b):
        for g, (u, v) in enumerate([(y, y), (X, y), (X, X)]):
            ref = math.fsum((u[:, j] * v[:, j]).tolist())
            assert abs(d[g * b + j] - ref) <= 1e-12 * float(np.sum(np.abs(u[:, j] * v[:, j]))), (j, g)
    Mx.close()


def _dos_tol(mu_h, b, E, s, c, kernel):
    # forward error of the three-term recurrence for T_m grows at worst like m^2 eps; bound
    # each energy's error by 4 eps nmom^2 times the sum of the absolute series terms
    mu2 = mu_h.reshape(-1, b).sum(axis=1)
    mt = mu2 / mu2[0]
    N = mt.shape[0]
    g = oracle.jackson(N) if kernel == "jackson" else np.ones(N)
    terms = np.abs(g * mt) * np.where(np.arange(N) == 0, 1.0, 2.0)
    x = (E - c) / s
    w = np.where(np.abs(x) < 1, np.pi * np.sqrt(np.maximum(1 - x * x, 1e-300)) * s, np.inf)
    return 4 * np.finfo(float).eps * N * N * terms.sum() / w


@pytest.mark.parametrize("b", [1, 8])
@pytest.mark.parametrize("kernel", ["jackson", "none"])
def test_kpm_dos_matches_oracle(sc, b, kernel):
    import torch

    A = synth.anderson3d(12)
    M = 60
    s, c = _scale(), 0.25
    Vd = dev(synth.block_vector(A.nrows, b, synth.SEED_X))
    Wd = torch.zeros_like(Vd)
    mu = torch.zeros((2 * M + 1) * b, dtype=torch.float64, device="cuda:0")
    Mx = sc.SellMatrix.from_csr(A, C=32, sigma=1)
    sc.sell_kpm(Mx, Vd, Wd, M, s, c, mu)
    E = np.concatenate([np.linspace(c - 1.1 * s, c + 1.1 * s, 333), [c - s, c + s, c]])
    rho = host(sc.sell_kpm_dos(mu, b, dev(E), s, c, kernel=kernel))
    mu_h = host(mu)
    ref = oracle.kpm_dos(mu_h, b, E, s, c, kernel=kernel)
    tol = _dos_tol(mu_h, b, E, s, c, kernel)
    assert np.all(np.abs(rho - ref) <= tol), np.max(np.abs(rho - ref) / np.where(tol > 0, tol, 1))
    assert np.all(rho[np.abs((E - c) / s) >= 1] == 0.0)
    Mx.close()


def test_kpm_dos_many_moments_and_edges(sc):
    # more moments than one LDS chunk holds (2048), two columns, synthetic moments
    import torch

    rng = np.random.default_rng(91)
    d = rng.uniform(-0.97, 0.97, 400)
    nmom, b = 5000, 2
    mom = np.cos(np.outer(np.arange(nmom), np.arccos(d))).mean(axis=1)
    mu_h = np.stack([0.7 * mom, 1.9 * mom], axis=1).ravel()
    E = np.linspace(-1.2, 1.2, 1001)
    rho = host(sc.sell_kpm_dos(dev(mu_h), b, dev(E), 1.0))
    ref = oracle.kpm_dos(mu_h, b, E, 1.0)
    assert np.all(np.abs(rho - ref) <= _dos_tol(mu_h, b, E, 1.0, 0.0, "jackson"))
    # one moment: the bare weight 1 / (pi sqrt(1 - x^2) s)
    one = host(sc.sell_kpm_dos(dev(np.array([3.0, 5.0])), 2, dev(E), 2.0))
    x = E / 2.0
    assert np.allclose(one, 1.0 / (np.pi * np.sqrt(1 - x * x) * 2.0), rtol=1e-14, atol=0)
    # no energies: nothing to do
    empty = torch.zeros(0, dtype=torch.float64, device="cuda:0")
    assert sc.sell_kpm_dos(dev(mu_h), b, empty, 1.0).numel() == 0
    for bad in (dict(s=0.0), dict(s=-1.0), dict(s=float("inf")), dict(c=float("nan"))):
        kw = dict(s=1.0, c=0.0)
        kw.update(bad)
        with pytest.raises(sc.SellError):
            sc.sell_kpm_dos(dev(mu_h), b, dev(E), kw["s"], kw["c"])
    with pytest.raises(sc.SellError):
        sc.sell_kpm_dos(dev(mu_h[:-1]), b, dev(E), 1.0)  # not whole rows of b moments


@pytest.mark.parametrize("b", [1, 8])
@pytest.mark.parametrize("N", [0, 1, 2, 60])
def test_cheb_filter_matches_oracle(sc, b, N):
    """Z = sum_m c_m T_m(A~) X with the chained accumulation of the augmented product. The
    three-term recurrence keeps |T_m(A~)| <= 1 on the scaled spectrum, so each step adds at most
    a few ulps of ||X|| per coefficient; the bound below allows 1e-13 N sum|c| ||X|| per column."""
    A = synth.anderson3d(10)
    s, c = _scale(), 0.3
    rng = np.random.default_rng(40 + N)
    coef = rng.normal(size=N + 1)
    X = synth.block_vector(A.nrows, b, synth.SEED_X)
    M = sc.SellMatrix.from_csr(A, C=32, sigma=1)
    Z = host(sc.sell_cheb_filter(M, dev(X), coef, s, c))
    ref = oracle.cheb_filter(A, X, coef, s, c)
    err = np.linalg.norm(Z - ref, axis=0)
    bound = 1e-13 * max(N, 1) * np.abs(coef).sum() * np.linalg.norm(X, axis=0)
    assert np.all(err <= bound), (err, bound)
    if N == 0:
        assert np.array_equal(Z, coef[0] * X)
    M.close()


def test_cheb_filter_exponential_f32_and_errors(sc):
    import scipy.special
    import torch

    A = synth.anderson3d(8)
    s = _scale()
    t, N = 2.0, 30
    coef = np.array([scipy.special.iv(m, t) * (1.0 if m == 0 else 2.0) for m in range(N + 1)])
    X = synth.block_vector(A.nrows, 4, 41)
    ref = oracle.cheb_filter(A, X, coef, s)  # exp(t A~) X, pinned against a dense expm
    # FP32 values and vectors: each step rounds to FP32 (relative 2^-24 per step of a stable
    # recurrence); the sum of |c_m| = e^t bounds the growth
    M32 = sc.SellMatrix.from_csr(A, C=32, sigma=1, dtype="f32")
    Z = host(sc.sell_cheb_filter(M32, dev(X, torch.float32), coef, s)).astype(np.float64)
    rel = np.linalg.norm(Z - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert rel.max() <= 50 * N * 2.0 ** -24 * np.abs(coef).sum(), rel
    Xd = dev(X)
    M = sc.SellMatrix.from_csr(A, C=32, sigma=1)
    with pytest.raises(sc.SellError):
        sc.sell_cheb_filter(M, Xd, coef, s, Z=Xd)  # Z must not be X
    with pytest.raises(sc.SellError):
        sc.sell_cheb_filter(M, Xd, coef, 0.0)
    with pytest.raises(sc.SellError):
        sc.sell_cheb_filter(M, Xd, [], s)
    M.close()
    M32.close()


def test_kpm_200_steps_within_fma_envelope(sc):
    """End to end over 200 steps (the benchmark's length): the GPU's v_200 and its 401 moments
    against the no-FMA oracle, within 10x the oracle's own spread between its FMA and no-FMA builds
    (plus 1e-15 of the norm). The moments come from the doubling identities on the GPU and from
    the direct recurrence to 400 in the oracle; measured, the GPU deviates 1.2x the spread for
    v_200 and 3.2x for the moments."""
    import torch

    A = synth.anderson3d(16)
    M, b = 200, 2
    s = _scale()
    V0 = synth.block_vector(A.nrows, b, synth.SEED_X)
    Vd = dev(V0)
    Wd = torch.zeros_like(Vd)
    mu = torch.zeros((2 * M + 1) * b, dtype=torch.float64, device="cuda:0")
    Mx = sc.SellMatrix.from_csr(A, C=32, sigma=1)
    last_in_w = sc.sell_kpm(Mx, Vd, Wd, M, s, 0.0, mu)
    mu_h = host(mu).reshape(2 * M + 1, b)
    vlast = host(Wd if last_in_w else Vd)
    Mx.close()
    for j in range(b):
        x = V0[:, j]
        _, v0 = oracle.chebyshev(A, x, M, s, 0.0)
        _, v1 = oracle.chebyshev(A, x, M, s, 0.0, fma=True)
        env_v = np.linalg.norm(v1 - v0)
        dv = np.linalg.norm(vlast[:, j] - v0)
        m0, _ = oracle.chebyshev(A, x, 2 * M, s, 0.0)
        m1, _ = oracle.chebyshev(A, x, 2 * M, s, 0.0, fma=True)
        env_mu = np.max(np.abs(m1 - m0))
        dmu = np.max(np.abs(mu_h[:, j] - m0))
        nx = float(x @ x)
        print(f"[envelope] column {j}: |v_gpu - v| = {dv:.3e}, FMA spread {env_v:.3e}; "
              f"moments {dmu:.3e}, FMA spread {env_mu:.3e}", flush=True)
        assert env_v > 0.0 and env_mu > 0.0  # the two builds do differ on this problem
        assert dv <= 10.0 * env_v + 1e-15 * np.linalg.norm(x), j
        assert dmu <= 10.0 * env_mu + 1e-15 * nx, j
