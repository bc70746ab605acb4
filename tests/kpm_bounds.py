"""Deterministic forward-error bounds of the Chebyshev recurrence and of the two ways of forming
its moments (direct, and by the doubling identities), used to compare two FP64 runs of the kernel
polynomial method that round differently (Sec. 5.3 names KPM as the user of the augmented
product; the recurrence and the identities are the textbook ones)."""
import numpy as np


def gamma_bound(k, u=2.0 ** -53):
    """gamma_k = k u / (1 - k u), the relative error bound of k rounded operations."""
    k = np.asarray(k, dtype=np.float64)
    return k * u / (1.0 - k * u)


def recurrence_bounds(A, nx, M, s, c):
    """Deterministic forward-error bounds D_m >= ||v^_m - v_m||_2, m = 0..M, for the Chebyshev
    recurrence v_1 = A~ v_0, v_{m+1} = 2 A~ v_m - v_{m-1}, A~ = (A - cI)/s, computed in FP64 in
    any order of summation, with or without fused multiply-adds, from ||v_0|| = nx.

    Local error of step m (row i, k_i stored entries): the row sum of k_i products, the shift, the
    scale and the subtraction of v_{m-1}, plus the rounding of the scale constant itself, give
    |e_m,i| <= gamma_{k_i+4} ((2/s)(|A| + |c|)|v^_m| + |v^_{m-1}|)_i, so
    ||e_m|| <= g (2 rho ||v^_m|| + ||v^_{m-1}||) with g = gamma_{max k + 4} and
    rho = (max_i sum_j |a_ij| + |c|)/s >= || |A~| ||_2 (|A| symmetric); step 0 has no v_{-1} and
    the factor 1 instead of 2.
    Propagation: d_m = v^_m - v_m obeys d_1 = e_0, d_{m+1} = 2 A~ d_m - d_{m-1} + e_m, whose
    solution is d_M = sum_{m<M} U_{M-1-m}(A~) e_m with U_k the Chebyshev polynomials of the second
    kind; ||U_k(A~)||_2 <= k + 1 on a symmetric A~ with spectrum in [-1, 1], hence
    D_M = sum_{m<M} (M - m) ||e_m||, and ||v^_m|| <= ||v_m|| + D_m <= nx + D_m."""
    lens = np.diff(A.rowptr)
    rows = np.bincount(np.repeat(np.arange(A.nrows), lens), weights=np.abs(A.val), minlength=A.nrows)
    rho = (float(rows.max()) + abs(c)) / s
    assert rho <= 1.0  # the scale bounds the spectrum
    g = float(gamma_bound(int(lens.max()) + 4))
    E, D = [], [0.0]
    for m in range(M):
        if m == 0:
            E.append(g * rho * nx)
        else:
            E.append(g * (2 * rho * (nx + D[m]) + nx + D[m - 1]))
        D.append(sum((m + 1 - j) * E[j] for j in range(m + 1)))
    return np.array(D)


def moment_bounds(D, nx, n):
    """Bounds on |mu^_k - mu_k|, k = 0..2M, for the two ways of forming the moments from the
    computed vectors (D from recurrence_bounds over 2M steps, nx = ||v_0||, n rows):
    direct, mu_k = <v_0, v_k>: nx D_k + gamma_n nx (nx + D_k);
    doubling, mu_2m = 2<v_m, v_m> - mu_0 and mu_2m+1 = 2<v_m+1, v_m> - mu_1:
      2 (nx (D_p + D_q) + D_p D_q) + 2 gamma_n (nx + D_p)(nx + D_q) + |mu^_0 or 1 - mu|
      + u (2 (nx + D_p)(nx + D_q) + nx^2), p and q the two indices of the product.
    Both hold for any order of summation of the dots (the GPU sums by a tree, the oracle with
    Neumaier compensation)."""
    u = 2.0 ** -53
    gn = float(gamma_bound(n))
    K = D.shape[0]
    direct = nx * D + gn * nx * (nx + D)
    dbl = np.zeros(K)
    dbl[0] = gn * nx * nx
    dbl[1] = nx * D[1] + gn * nx * (nx + D[1])
    for k in range(2, K):
        p, q = (k // 2, k // 2) if k % 2 == 0 else ((k - 1) // 2, (k + 1) // 2)
        vp, vq = nx + D[p], nx + D[q]
        dbl[k] = (2 * (nx * (D[p] + D[q]) + D[p] * D[q]) + 2 * gn * vp * vq + dbl[k % 2]
                  + u * (2 * vp * vq + nx * nx))
    return direct, dbl
