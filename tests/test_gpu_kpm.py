"""GPU parity of the kernel polynomial method recurrence (sell_kpm) and of one augmented
product at the full size of the 128^3 Anderson workload."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import abs_product, colwise_relerr, dev, gamma_bound, host
from kpm_bounds import moment_bounds, recurrence_bounds

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


@pytest.fixture(scope="module")
def anderson128():
    return synth.anderson3d(128)


def _kpm_step_check(A, got_y, got_d, X, Y0, ref, what, dots=(0, 1)):
    """One augmented KPM product on the whole output against the oracle applied to the same
    inputs: every element within 2 gamma_{k+4} of its error scale (each side's bound for k stored
    entries, then shift, scale and axpby, and the rounding of the scale constant), the normwise
    relative error of
    every column within 1e-12, and the requested dots within 1e-12 sum |u_i v_i|."""
    ry, _, rd = ref
    k = A.row_lengths().reshape(-1, 1)
    scale = what["scale"]
    bad = np.abs(got_y - ry) > 2 * gamma_bound(k + 4) * scale
    assert not bad.any(), (what["name"], int(bad.sum()))
    assert colwise_relerr(got_y, ry) <= 1e-12, what["name"]
    b = X.shape[1]
    pairs = [(ry, ry), (X, ry), (X, X)]
    for g in dots:
        u, v = pairs[g]
        seg = slice(g * b, (g + 1) * b)
        assert np.all(np.abs(got_d[seg] - rd[seg]) <= 1e-12 * np.sum(np.abs(u * v), axis=0)), (what["name"], g)


@pytest.mark.parametrize("b", [1, 8])
def test_full_size_anderson_128_whole_output(sc, anderson128, b):
    """The workload the benchmark times (128^3 periodic Anderson, n = 2,097,152, SELL-32-1): one
    augmented product of the KPM recurrence (alpha = 2/s, beta = -1, all three dots), the whole
    output compared with the oracle element by element."""
    import torch

    A = anderson128
    s = _scale()
    Mx = sc.SellMatrix.from_csr(A, C=32, sigma=1)
    X = synth.block_vector(A.nrows, b, synth.SEED_X)
    Y0 = synth.block_vector(A.nrows, b, synth.SEED_Y)
    Xd, Yd = dev(X), dev(Y0)
    dot = torch.zeros(3 * b, dtype=torch.float64, device="cuda:0")
    alpha = 2.0 / s
    sc.sell_spmmv_aug(Mx, Xd, Yd, flags=sc.SCALE | sc.SHIFT | sc.AXPBY | sc.DOTS, alpha=alpha, gamma=0.0,
                      beta=-1.0, dot=dot)
    got, d = host(Yd), host(dot)
    Mx.close()
    ref = oracle.spmmv_aug(A, X, Y=Y0, flags=oracle.SCALE | oracle.SHIFT | oracle.AXPBY | oracle.DOT_YY
                           | oracle.DOT_XY | oracle.DOT_XX, alpha=alpha, gamma=0.0, beta=-1.0)
    scale = alpha * abs_product(A, X) + np.abs(Y0)
    _kpm_step_check(A, got, d, X, Y0, ref, dict(name=f"b={b}", scale=scale), dots=(0, 1, 2))


def test_full_size_anderson_128_kpm_three_steps(sc, anderson128):
    """Three steps of the benchmark's KPM recurrence at full size and b = 8, each step's whole
    output compared with the oracle applied to the same device input (step-local parity), then
    sell_kpm over the same three steps: its v_3 equal bit for bit to the step-by-step products
    (the same kernels on the same inputs), and its seven moments within the forward-error bounds
    of the oracle's direct recurrence."""
    import torch

    A = anderson128
    s = _scale()
    b = 8
    Mx = sc.SellMatrix.from_csr(A, C=32, sigma=1)
    V0 = synth.block_vector(A.nrows, b, synth.SEED_X)
    x = dev(V0)
    y = torch.zeros_like(x)
    dot = torch.zeros(3 * b, dtype=torch.float64, device="cuda:0")
    for step in range(3):
        xin, yin = host(x), host(y)
        if step == 0:
            fl, ofl, kw = (sc.SCALE | sc.SHIFT | sc.DOTS, oracle.SCALE | oracle.SHIFT | oracle.DOT_YY
                           | oracle.DOT_XY | oracle.DOT_XX, dict(alpha=1.0 / s, gamma=0.0, beta=0.0))
        else:
            fl, ofl, kw = (sc.SCALE | sc.SHIFT | sc.AXPBY | sc.DOT_YY | sc.DOT_XY, oracle.SCALE | oracle.SHIFT
                           | oracle.AXPBY | oracle.DOT_YY | oracle.DOT_XY, dict(alpha=2.0 / s, gamma=0.0, beta=-1.0))
        sc.sell_spmmv_aug(Mx, x, y, flags=fl, dot=dot, **kw)
        ref = oracle.spmmv_aug(A, xin, Y=yin, flags=ofl, **kw)
        scale = kw["alpha"] * abs_product(A, xin) + abs(kw["beta"]) * np.abs(yin)
        _kpm_step_check(A, host(y), host(dot), xin, yin, ref, dict(name=f"step {step}", scale=scale),
                        dots=(0, 1, 2) if step == 0 else (0, 1))
        x, y = y, x
    v3 = host(x)
    mu = torch.zeros(7 * b, dtype=torch.float64, device="cuda:0")
    Vd, Wd = dev(V0), torch.zeros_like(x)
    last_in_w = sc.sell_kpm(Mx, Vd, Wd, 3, s, 0.0, mu)
    assert np.array_equal(host(Wd if last_in_w else Vd), v3)
    mu_h = host(mu).reshape(7, b)
    Mx.close()
    for j in range(b):
        nx = float(np.linalg.norm(V0[:, j]))
        D = recurrence_bounds(A, nx, 6, s, 0.0)
        direct, dbl = moment_bounds(D, nx, A.nrows)
        m0, _ = oracle.chebyshev(A, V0[:, j], 6, s, 0.0)
        assert np.all(np.abs(mu_h[:, j] - m0) <= direct + dbl), j


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


def test_kpm_200_steps_within_derived_bound(sc):
    """End to end over 200 steps (the benchmark's length): the GPU's v_200 and its 401 moments
    against the no-FMA oracle, within the sum of the two sides' deterministic forward-error bounds
    (kpm_bounds.recurrence_bounds and moment_bounds). The GPU forms the moments from the doubling
    identities, the oracle by the direct recurrence to 400 steps. The oracle's own FMA/no-FMA spread is
    printed beside it, as a sample of the rounding noise (not a bound)."""
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
        nx = float(np.linalg.norm(x))
        D = recurrence_bounds(A, nx, 2 * M, s, 0.0)
        direct, dbl = moment_bounds(D, nx, A.nrows)
        _, v0 = oracle.chebyshev(A, x, M, s, 0.0)
        _, v1 = oracle.chebyshev(A, x, M, s, 0.0, fma=True)
        env_v = np.linalg.norm(v1 - v0)
        dv = np.linalg.norm(vlast[:, j] - v0)
        m0, _ = oracle.chebyshev(A, x, 2 * M, s, 0.0)
        m1, _ = oracle.chebyshev(A, x, 2 * M, s, 0.0, fma=True)
        env_mu = np.max(np.abs(m1 - m0))
        dmu = np.abs(mu_h[:, j] - m0)
        bmu = direct + dbl
        print(f"[kpm 200] column {j}: |v_gpu - v| = {dv:.3e} (bound {2 * D[M]:.3e}, FMA spread {env_v:.3e}); "
              f"moments max {dmu.max():.3e} (max ratio to bound {np.max(dmu / bmu):.2e}, "
              f"FMA spread {env_mu:.3e})", flush=True)
        assert dv <= 2 * D[M], j
        assert np.all(dmu <= bmu), (j, int(np.argmax(dmu / bmu)))
