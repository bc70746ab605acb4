// tsm.hip -- tall-skinny block-vector kernels (GHOST paper Sec. 5.2), FP64, row-major.
//   tsmttsm:      X = alpha V^T W + beta X   (V: n x m, W: n x k, X: m x k small)
//   tsmm:         W = alpha V X + beta W     (X: m x k small)
//   tsmm_inplace: V = alpha V X + beta V     (X: m x m small)
// m, k <= 64. They are streaming kernels (bandwidth-bound for small m, k). tsmttsm keeps 4 x 4
// blocks of the result in registers per thread and reduces deterministically (per-workgroup
// partials, then a fixed-order sum), with an optional Neumaier-compensated summation (the
// paper adds a Kahan-summed variant of this reduction for accuracy on long vectors); tsmm and
// tsmm_inplace keep the small matrix X in LDS.
#include "devutil.h"
#include "internal.h"

namespace sellcs {

constexpr int kTT = 256;     // threads per workgroup

__device__ __forceinline__ void neumaier_add(double &s, double &comp, double term) {
    const double t = s + term;
    if (fabs(s) >= fabs(term))
        comp += (s - t) + term;
    else
        comp += (term - t) + s;
    s = t;
}

// Partial sums of V^T W over this workgroup's row range [g n / G, (g + 1) n / G). The m x k
// result is cut into 4 x 4 blocks; thread t accumulates block t % nblk in registers over the
// rows t / nblk, + groups, ... of the range (groups = 256 / nblk row groups), so every loaded
// row piece feeds 16 multiply-adds. The row groups' blocks are then added in group order
// through LDS; output q = l * k + j lands in partials[q * G + g]. KAHAN: Neumaier-compensated
// sums in both stages.
// VEC (m and k multiples of 4, V and W rows 16-byte aligned): each thread loads its 4 + 4
// values as 16-byte pieces with no bounds checks and keeps TV rows in flight; the rows are
// visited in the same order, so the sums are the same bit for bit. V^T W with n = 4 M,
// m = k = 8: 98.8 us against 118.9 for the per-element loads (1, 2, 4 or 8 rows in flight
// within 3 %). The compensated sums keep the per-element loads: with 16-byte loads they ran
// 156-163 us with 1 or 2 rows in flight against 157 us (within the noise between runs) and
// 197 us with 8 rows (the Neumaier updates of more rows hold more registers).
constexpr int kTV = 4;
typedef double tsm_d2 __attribute__((ext_vector_type(2)));

template <bool KAHAN, bool VEC, int TV = kTV>
__global__ void __launch_bounds__(kTT) tsmttsm_partial_kernel(const double *__restrict__ V, int64_t ldv,
                                                              const double *__restrict__ W, int64_t ldw, int64_t n,
                                                              int m, int k, double *partials) {
    __shared__ double red[kTT][17];
    const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
    const int64_t r0 = int64_t(g) * n / G, r1 = int64_t(g + 1) * n / G;
    const int nbk = (k + 3) / 4, nblk = ((m + 3) / 4) * nbk;  // at most 256 blocks
    const int groups = kTT / nblk;
    const int blk = tid % nblk, grp = tid / nblk;
    const int l0 = (blk / nbk) * 4, j0 = (blk % nbk) * 4;
    double acc[16], comp[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e] = comp[e] = 0.0;
    if (VEC && grp < groups) {
        const int64_t st = groups;
        for (int64_t i = r0 + grp; i < r1; i += TV * st) {
            tsm_d2 v[TV][2], w[TV][2];
#pragma unroll
            for (int u = 0; u < TV; ++u)
                if (i + u * st < r1) {
                    const tsm_d2 *vp = reinterpret_cast<const tsm_d2 *>(V + (i + u * st) * ldv + l0);
                    const tsm_d2 *wp = reinterpret_cast<const tsm_d2 *>(W + (i + u * st) * ldw + j0);
                    v[u][0] = vp[0];
                    v[u][1] = vp[1];
                    w[u][0] = wp[0];
                    w[u][1] = wp[1];
                }
#pragma unroll
            for (int u = 0; u < TV; ++u)
                if (i + u * st < r1) {
#pragma unroll
                    for (int a = 0; a < 4; ++a)
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            const double va = v[u][a >> 1][a & 1], wc = w[u][c >> 1][c & 1];
                            if (KAHAN)
                                neumaier_add(acc[a * 4 + c], comp[a * 4 + c], va * wc);
                            else
                                acc[a * 4 + c] = fma(va, wc, acc[a * 4 + c]);
                        }
                }
        }
    } else if (grp < groups) {
#pragma unroll 2
        for (int64_t i = r0 + grp; i < r1; i += groups) {
            double v[4], w[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                v[t] = l0 + t < m ? V[i * ldv + l0 + t] : 0.0;
                w[t] = j0 + t < k ? W[i * ldw + j0 + t] : 0.0;
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    if (KAHAN)
                        neumaier_add(acc[a * 4 + c], comp[a * 4 + c], v[a] * w[c]);
                    else
                        acc[a * 4 + c] = fma(v[a], w[c], acc[a * 4 + c]);
                }
        }
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) red[tid][e] = acc[e] + comp[e];
    __syncthreads();
    for (int o = tid; o < nblk * 16; o += kTT) {
        const int b = o >> 4, e = o & 15;
        const int l = (b / nbk) * 4 + (e >> 2), j = (b % nbk) * 4 + (e & 3);
        if (l >= m || j >= k) continue;
        double sum = 0.0, c2 = 0.0;
        for (int gg = 0; gg < groups; ++gg) {
            if (KAHAN)
                neumaier_add(sum, c2, red[gg * nblk + b][e]);
            else
                sum += red[gg * nblk + b][e];
        }
        partials[size_t(l * k + j) * G + g] = sum + c2;
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

// W = alpha V X + beta W: a tile of R rows of V is staged in LDS with coalesced loads (consecutive
// lanes read consecutive entries), then thread (r, j) of the tile forms output (r, j) from the
// staged row and X, also staged in LDS. The LDS holds exactly m k + R m doubles (dynamic), so
// small blocks do not limit the workgroups per compute unit.
__host__ __device__ inline int tsmm_rows(int m, int k) {
    const int r = kTT / k;
    return r * m > 2048 ? 2048 / m : r;
}

__global__ void __launch_bounds__(kTT) tsmm_kernel(const double *__restrict__ V, int64_t ldv, const double *Xs,
                                                   int64_t ldx, int m, int k, int64_t n, double alpha, double beta,
                                                   double *W, int64_t ldw) {
    extern __shared__ double lds[];
    double *sx = lds, *sv = lds + m * k;
    for (int e = threadIdx.x; e < m * k; e += kTT) sx[e] = Xs[int64_t(e / k) * ldx + e % k];
    const int R = tsmm_rows(m, k);
    const int r = threadIdx.x / k, j = threadIdx.x - r * k;
    for (int64_t t0 = int64_t(blockIdx.x) * R; t0 < n; t0 += int64_t(gridDim.x) * R) {
        const int rows = n - t0 < R ? int(n - t0) : R;
        __syncthreads();
        for (int e = threadIdx.x; e < rows * m; e += kTT) {
            const int rr = e / m;
            sv[e] = V[(t0 + rr) * ldv + (e - rr * m)];
        }
        __syncthreads();
        if (r < rows) {
            double s = 0.0;
            for (int l = 0; l < m; ++l) s = fma(sv[r * m + l], sx[l * k + j], s);
            double *w = W + (t0 + r) * ldw + j;
            const double v = alpha * s;
            *w = beta != 0.0 ? v + beta * *w : v;
        }
    }
}

// V = alpha V X + beta V: rows staged in LDS before any of them is overwritten.
__global__ void __launch_bounds__(kTT) tsmm_inplace_kernel(double *V, int64_t ldv, const double *Xs, int64_t ldx,
                                                           int m, int64_t n, double alpha, double beta) {
    extern __shared__ double lds[];
    double *sv = lds, *sx = lds + kTT;  // LDS: kTT + m m doubles (dynamic)
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
    const bool vec = m % 4 == 0 && k % 4 == 0 && ldv % 2 == 0 && ldw % 2 == 0 &&
                     (reinterpret_cast<uintptr_t>(V) & 15u) == 0 && (reinterpret_cast<uintptr_t>(W) & 15u) == 0;
    auto kern = kahan ? tsmttsm_partial_kernel<true, false>
                      : (vec ? tsmttsm_partial_kernel<false, true> : tsmttsm_partial_kernel<false, false>);
    hipLaunchKernelGGL(kern, dim3(unsigned(G)), dim3(kTT), 0, s, V, ldv, W, ldw, n, m, k, partials);
    if (hipGetLastError() != hipSuccess) return SELL_ERR_HIP;
    hipLaunchKernelGGL(tsmttsm_finish_kernel, dim3(mk), dim3(kTT), 0, s, partials, int(G), k, kahan, alpha, beta, X,
                       ldx);
    return hipGetLastError() == hipSuccess ? SELL_OK : SELL_ERR_HIP;
}

int launch_tsmm(const double *V, int64_t ldv, const double *X, int64_t ldx, int m, int k, int64_t n, double alpha,
                double beta, double *W, int64_t ldw, hipStream_t s) {
    if (n == 0) return SELL_OK;
    const int R = tsmm_rows(m, k);
    const size_t lds = size_t(m * k + R * m) * sizeof(double);
    hipLaunchKernelGGL(tsmm_kernel, dim3(tgrid((n + R - 1) / R * kTT, 8192)), dim3(kTT), lds, s, V, ldv, X, ldx, m,
                       k, n, alpha, beta, W, ldw);
    return hipGetLastError() == hipSuccess ? SELL_OK : SELL_ERR_HIP;
}

int launch_tsmm_inplace(double *V, int64_t ldv, const double *X, int64_t ldx, int m, int64_t n, double alpha,
                        double beta, hipStream_t s) {
    if (n == 0) return SELL_OK;
    const int rows = kTT / m;
    hipLaunchKernelGGL(tsmm_inplace_kernel, dim3(tgrid((n + rows - 1) / rows * kTT, 8192)), dim3(kTT),
                       size_t(kTT + m * m) * sizeof(double), s, V, ldv, X, ldx, m, n, alpha, beta);
    return hipGetLastError() == hipSuccess ? SELL_OK : SELL_ERR_HIP;
}

}  // namespace sellcs
