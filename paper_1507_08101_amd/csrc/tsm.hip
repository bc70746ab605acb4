// tsm.hip -- tall-skinny block-vector kernels (GHOST paper Sec. 5.2), FP64, row-major.
//   tsmttsm:      X = alpha V^T W + beta X   (V: n x m, W: n x k, X: m x k small)
//   tsmm:         W = alpha V X + beta W     (X: m x k small)
//   tsmm_inplace: V = alpha V X + beta V     (X: m x m small)
// m, k <= 64. They are streaming kernels (bandwidth-bound for small m, k): rows are staged
// through LDS with coalesced loads, the small matrix X sits in LDS. The inner product
// tsmttsm reduces deterministically (per-workgroup partials, then a fixed-order sum), with an
// optional Neumaier-compensated summation (the paper adds a Kahan-summed variant of this
// reduction for accuracy on long vectors).
#include "devutil.h"
#include "internal.h"

namespace sellcs {

constexpr int kTT = 256;     // threads per workgroup
constexpr int kRowTile = 32; // rows staged per LDS tile in tsmttsm

__device__ __forceinline__ void neumaier_add(double &s, double &comp, double term) {
    const double t = s + term;
    if (fabs(s) >= fabs(term))
        comp += (s - t) + term;
    else
        comp += (term - t) + s;
    s = t;
}

// Partial sums of V^T W over this workgroup's row range; output entry q = l * k + j is
// handled by threads q, q + 256, ...; partials[q * G + g].
__global__ void __launch_bounds__(kTT) tsmttsm_partial_kernel(const double *__restrict__ V, int64_t ldv,
                                                              const double *__restrict__ W, int64_t ldw, int64_t n,
                                                              int m, int k, int kahan, double *partials) {
    __shared__ double sv[kRowTile][64];
    __shared__ double sw[kRowTile][64];
    const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
    const int64_t r0 = int64_t(g) * n / G, r1 = int64_t(g + 1) * n / G;
    const int mk = m * k;
    constexpr int QPT = (64 * 64 + kTT - 1) / kTT;  // outputs per thread at most
    double s[QPT], comp[QPT];
#pragma unroll
    for (int u = 0; u < QPT; ++u) s[u] = comp[u] = 0.0;
    for (int64_t t0 = r0; t0 < r1; t0 += kRowTile) {
        const int rows = int(min<int64_t>(kRowTile, r1 - t0));
        __syncthreads();
        for (int e = tid; e < rows * m; e += kTT) sv[e / m][e % m] = V[(t0 + e / m) * ldv + e % m];
        for (int e = tid; e < rows * k; e += kTT) sw[e / k][e % k] = W[(t0 + e / k) * ldw + e % k];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < QPT; ++u) {
            const int q = tid + u * kTT;
            if (q < mk) {
                const int l = q / k, j = q - l * k;
                for (int r = 0; r < rows; ++r) {
                    const double term = sv[r][l] * sw[r][j];
                    if (kahan)
                        neumaier_add(s[u], comp[u], term);
                    else
                        s[u] += term;
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < QPT; ++u) {
        const int q = tid + u * kTT;
        if (q < mk) partials[size_t(q) * G + g] = s[u] + comp[u];
    }
}

// X[q] = alpha * sum_g partials[q * G + g] + beta * X[q], one workgroup per entry.
__global__ void __launch_bounds__(kTT) tsmttsm_finish_kernel(const double *partials, int G, int k, int kahan,
                                                             double alpha, double beta, double *X, int64_t ldx) {
    const int q = blockIdx.x;
    const double *p = partials + size_t(q) * G;
    double s = 0.0, comp = 0.0;
    for (int t = threadIdx.x; t < G; t += kTT) {
        if (kahan)
            neumaier_add(s, comp, p[t]);
        else
            s += p[t];
    }
    const double tot = block_sum_256(s) + block_sum_256(comp);
    if (threadIdx.x == 0) {
        const int l = q / k, j = q - l * k;
        double *x = X + int64_t(l) * ldx + j;
        const double v = alpha * tot;
        *x = beta != 0.0 ? v + beta * *x : v;
    }
}

// W = alpha V X + beta W: one thread per output element; X staged in LDS.
__global__ void __launch_bounds__(kTT) tsmm_kernel(const double *__restrict__ V, int64_t ldv, const double *Xs,
                                                   int64_t ldx, int m, int k, int64_t n, double alpha, double beta,
                                                   double *W, int64_t ldw) {
    __shared__ double sx[64 * 64];
    for (int e = threadIdx.x; e < m * k; e += kTT) sx[e] = Xs[int64_t(e / k) * ldx + e % k];
    __syncthreads();
    const int64_t N = n * k;
    for (int64_t e = int64_t(blockIdx.x) * kTT + threadIdx.x; e < N; e += int64_t(gridDim.x) * kTT) {
        const int64_t i = e / k;
        const int j = int(e - i * k);
        const double *v = V + i * ldv;
        double s = 0.0;
        for (int l = 0; l < m; ++l) s += v[l] * sx[l * k + j];
        double *w = W + i * ldw + j;
        const double r = alpha * s;
        *w = beta != 0.0 ? r + beta * *w : r;
    }
}

// V = alpha V X + beta V: rows staged in LDS before any of them is overwritten.
__global__ void __launch_bounds__(kTT) tsmm_inplace_kernel(double *V, int64_t ldv, const double *Xs, int64_t ldx,
                                                           int m, int64_t n, double alpha, double beta) {
    __shared__ double sx[64 * 64];
    __shared__ double sv[kTT];
    for (int e = threadIdx.x; e < m * m; e += kTT) sx[e] = Xs[int64_t(e / m) * ldx + e % m];
    const int rows = kTT / m;  // rows per tile
    for (int64_t t0 = int64_t(blockIdx.x) * rows; t0 < n; t0 += int64_t(gridDim.x) * rows) {
        const int r = threadIdx.x / m, j = threadIdx.x - (threadIdx.x / m) * m;
        const bool act = r < rows && t0 + r < n;
        __syncthreads();
        if (act) sv[r * m + j] = V[(t0 + r) * ldv + j];
        __syncthreads();
        if (act) {
            double s = 0.0;
            for (int l = 0; l < m; ++l) s += sv[r * m + l] * sx[l * m + j];
            const double v = alpha * s;
            V[(t0 + r) * ldv + j] = beta != 0.0 ? v + beta * sv[r * m + j] : v;
        }
    }
}

static unsigned tgrid(int64_t work, unsigned cap) {
    int64_t g = (work + kTT - 1) / kTT;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return unsigned(g);
}

int launch_tsmttsm(const double *V, int64_t ldv, const double *W, int64_t ldw, int64_t n, int m, int k, double alpha,
                   double beta, double *X, int64_t ldx, int kahan, double *partials, int64_t max_partials,
                   hipStream_t s) {
    const int mk = m * k;
    int64_t G = (n + 63) / 64;
    if (G > 1024) G = 1024;
    if (G > max_partials / mk) G = max_partials / mk;
    if (G < 1) G = 1;
    hipLaunchKernelGGL(tsmttsm_partial_kernel, dim3(unsigned(G)), dim3(kTT), 0, s, V, ldv, W, ldw, n, m, k, kahan,
                       partials);
    if (hipGetLastError() != hipSuccess) return SELL_ERR_HIP;
    hipLaunchKernelGGL(tsmttsm_finish_kernel, dim3(mk), dim3(kTT), 0, s, partials, int(G), k, kahan, alpha, beta, X,
                       ldx);
    return hipGetLastError() == hipSuccess ? SELL_OK : SELL_ERR_HIP;
}

int launch_tsmm(const double *V, int64_t ldv, const double *X, int64_t ldx, int m, int k, int64_t n, double alpha,
                double beta, double *W, int64_t ldw, hipStream_t s) {
    if (n == 0) return SELL_OK;
    hipLaunchKernelGGL(tsmm_kernel, dim3(tgrid(n * k, 8192)), dim3(kTT), 0, s, V, ldv, X, ldx, m, k, n, alpha, beta,
                       W, ldw);
    return hipGetLastError() == hipSuccess ? SELL_OK : SELL_ERR_HIP;
}

int launch_tsmm_inplace(double *V, int64_t ldv, const double *X, int64_t ldx, int m, int64_t n, double alpha,
                        double beta, hipStream_t s) {
    if (n == 0) return SELL_OK;
    const int rows = kTT / m;
    hipLaunchKernelGGL(tsmm_inplace_kernel, dim3(tgrid((n + rows - 1) / rows * kTT, 8192)), dim3(kTT), 0, s, V, ldv,
                       X, ldx, m, n, alpha, beta);
    return hipGetLastError() == hipSuccess ? SELL_OK : SELL_ERR_HIP;
}

}  // namespace sellcs
