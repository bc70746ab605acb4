"""Pins of the oracle's KPM density-of-states reconstruction (textbook kernel polynomial
method; the paper names KPM as a user of the fused block product but does not define it):
the Jackson factors against their construction as an autocorrelation, the reconstruction
against Chebyshev orthogonality under Gauss-Chebyshev quadrature, positivity of the Jackson
density against the Gibbs oscillations of the undamped one, and the closed-form density of
states of the periodic chain."""
import numpy as np
import pytest

import oracle
import synth


@pytest.mark.parametrize("N", [1, 2, 5, 50, 401])
def test_jackson_is_autocorrelation_of_sine_window(N):
    # the optimal positive kernel: g_n = sum_v a_v a_{v+n} with a_v ~ sin(pi (v + 1) / (N + 1)), |a| = 1
    a = np.sin(np.pi * (np.arange(N) + 1) / (N + 1))
    a /= np.linalg.norm(a)
    ref = np.array([np.dot(a[: N - n], a[n:]) for n in range(N)])
    g = oracle.jackson(N)
    assert g.shape == (N,)
    assert abs(g[0] - 1.0) <= 1e-15
    assert np.abs(g - ref).max() <= 1e-14


def _diag_moments(d, N):
    # exact normalised Chebyshev moments of the spectral measure of diag(d): mean_i T_m(d_i)
    th = np.arccos(d)
    return np.cos(np.outer(np.arange(N), th)).mean(axis=1)


@pytest.mark.parametrize("kernel", ["jackson", "none"])
@pytest.mark.parametrize("s,c", [(1.0, 0.0), (3.5, -0.75)])
def test_dos_chebyshev_orthogonality(kernel, s, c):
    rng = np.random.default_rng(5)
    N, b = 37, 3
    d = np.concatenate([rng.uniform(-0.9, -0.4, 300), rng.uniform(0.2, 0.95, 200)])
    mu1 = _diag_moments(d, N)
    # a block of b "columns" whose sums give the moments times a positive weight
    w = np.array([0.5, 1.25, 2.0])
    mu = np.outer(mu1, w).ravel()
    K = 2 * N + 7
    xk = np.cos(np.pi * (np.arange(K) + 0.5) / K)
    rho = oracle.kpm_dos(mu, b, c + s * xk, s, c, kernel=kernel)
    f = rho * np.pi * np.sqrt(1 - xk * xk) * s  # the Chebyshev series itself
    g = oracle.jackson(N) if kernel == "jackson" else np.ones(N)
    for m in range(N + 5):
        got = np.mean(f * np.cos(m * np.arccos(xk)))
        want = g[m] * mu1[m] if m < N else 0.0
        assert abs(got - want) <= 1e-13, (m, got, want)


def test_jackson_density_is_nonnegative_undamped_oscillates():
    rng = np.random.default_rng(6)
    d = np.concatenate([rng.uniform(-0.8, -0.6, 500), np.full(100, 0.3), rng.uniform(0.5, 0.55, 400)])
    N = 120
    mu = _diag_moments(d, N)
    E = np.linspace(-0.999, 0.999, 4001)
    rj = oracle.kpm_dos(mu, 1, E, 1.0)
    rn = oracle.kpm_dos(mu, 1, E, 1.0, kernel="none")
    assert rj.min() >= -1e-12 * rj.max()
    assert rn.min() < -0.01 * rn.max()  # Gibbs oscillations without damping
    # both integrate to one (trapezoid on a fine grid of the smooth Jackson density)
    assert abs(np.trapezoid(rj, E) - 1.0) < 2e-3


def test_dos_outside_band_is_zero():
    mu = _diag_moments(np.array([0.1, -0.2]), 10)
    r = oracle.kpm_dos(mu, 1, np.array([-5.0, -2.0, 2.0, 7.0, 2.0 + 1e-12]), 2.0)
    assert np.all(r == 0.0)


def test_periodic_chain_closed_form():
    # tight-binding ring: eigenvalues 2 cos(2 pi k / n), density of states 1 / (pi sqrt(4 - E^2))
    n, s, N = 4096, 2.2, 400
    lam = 2 * np.cos(2 * np.pi * np.arange(n) / n)
    mu = _diag_moments(lam / s, N)
    E = np.array([-1.0, 0.0, 0.5, 1.0, 1.5])
    rho = oracle.kpm_dos(mu, 1, E, s)
    exact = 1.0 / (np.pi * np.sqrt(4 - E * E))
    assert np.abs(rho / exact - 1).max() < 0.01


def test_stochastic_block_moments_of_the_chain():
    # moments from the oracle's own recurrence on random starting vectors, averaged over the block
    n, s, M, b = 65536, 2.2, 100, 8
    rowptr = np.arange(0, 2 * n + 1, 2, dtype=np.int64)
    i = np.arange(n)
    cols = np.sort(np.stack([(i - 1) % n, (i + 1) % n], axis=1), axis=1).ravel().astype(np.int32)
    A = synth.CSR(n, n, rowptr, cols, np.ones(2 * n), "ring")
    V = synth.block_vector(n, b, 77)
    mu = np.empty((2 * M + 1, b))
    for j in range(b):
        mj, _ = oracle.chebyshev(A, np.ascontiguousarray(V[:, j]), 2 * M, s)
        mu[:, j] = mj
    E = np.array([-1.0, 0.0, 1.0])
    rho = oracle.kpm_dos(mu.ravel(), b, E, s)
    # against the exact moments of the same ring at the same order: the block average is a
    # stochastic trace estimate with an error of about 1 / sqrt(n b) per moment, so the series
    # f = rho pi sqrt(1 - x^2) s is off by about 2 |g| / sqrt(n b); allow four times that
    lam = 2 * np.cos(2 * np.pi * np.arange(n) / n)
    ref = oracle.kpm_dos(_diag_moments(lam / s, 2 * M + 1), 1, E, s)
    x = E / s
    w = np.pi * np.sqrt(1 - x * x) * s
    sigma_f = 2 * np.linalg.norm(oracle.jackson(2 * M + 1)) / np.sqrt(n * b)
    assert np.all(np.abs(rho - ref) * w <= 4 * sigma_f), (rho, ref, sigma_f)
    assert np.all(np.abs(rho - ref) * w > 0)  # a real estimate, not the exact moments


def test_recurrence_bounds_hold_between_oracle_builds():
    """The forward-error bounds that judge the GPU's 200-step KPM against the oracle
    (kpm_bounds) must hold between any two correct FP64 runs: the oracle's no-FMA and FMA builds
    (v_M within 2 D_M, direct moments within twice the direct bound) and, on the oracle's own
    vectors, the doubling-identity moments against the direct ones (within the sum of both
    bounds). The bounds must also be non-trivial: well below the size of the quantities."""
    from kpm_bounds import moment_bounds, recurrence_bounds

    A = synth.anderson3d(8)
    s = (6 + 16.5 / 2) / 0.99
    M = 60
    x = synth.block_vector(A.nrows, 1, 9)[:, 0]
    nx = float(np.linalg.norm(x))
    D = recurrence_bounds(A, nx, 2 * M, s, 0.0)
    direct, dbl = moment_bounds(D, nx, A.nrows)
    assert D[2 * M] < 1e-9 * nx and np.all(np.diff(D) >= 0)
    mu0, v0 = oracle.chebyshev(A, x, M, s, 0.0)
    mu1, v1 = oracle.chebyshev(A, x, M, s, 0.0, fma=True)
    assert np.linalg.norm(v1 - v0) <= 2 * D[M]
    m0, _ = oracle.chebyshev(A, x, 2 * M, s, 0.0)
    m1, _ = oracle.chebyshev(A, x, 2 * M, s, 0.0, fma=True)
    assert np.all(np.abs(m1 - m0) <= 2 * direct)
    vs = [x] + [oracle.chebyshev(A, x, m, s, 0.0)[1] for m in range(1, M + 1)]
    dbl_mu = np.zeros(2 * M + 1)
    dbl_mu[0], dbl_mu[1] = x @ x, x @ vs[1]
    for m in range(1, M + 1):
        dbl_mu[2 * m] = 2 * (vs[m] @ vs[m]) - dbl_mu[0]
        if 2 * m + 1 <= 2 * M:
            dbl_mu[2 * m + 1] = 2 * (vs[m + 1] @ vs[m]) - dbl_mu[1]
    assert np.all(np.abs(dbl_mu - m0) <= direct + dbl)
    # a dropped term is caught: the recurrence without the - v_{m-1} is far outside the bound
    wrong = [x, vs[1]]
    for m in range(1, M):
        wrong.append(2 * oracle.spmmv(A, wrong[m].reshape(-1, 1))[:, 0] / s)
    assert np.linalg.norm(wrong[M] - v0) > 1e3 * D[M]
