// grad.hip -- kernels for derivatives with respect to the stored matrix values.
//
// For a product Y = A X the gradient of a scalar loss with respect to the value of stored
// entry p = (i, k) is sum_j G[i, j] X[k, j] with G = dL/dY: an outer product restricted to
// the sparsity pattern. It is accumulated here in SELL-C-sigma order (entry k of slot r of
// chunk c at cs[c] + k*C + r), so consecutive lanes touch consecutive addresses, and mapped
// to the caller's CSR order once at the end.
#include "convert.h"
#include "internal.h"

namespace sellcs {

// dsell[e] += alpha * sum_j G[row(e), j] X[col(e), j] for every real entry e of the tiles of
// this workgroup; one lane per row slot, columns summed in order.
template <class TX>
__global__ void __launch_bounds__(256) grad_accum_kernel(const int32_t *__restrict__ col, const int32_t *cl,
                                                         const int64_t *cs, const int32_t *perm, int64_t nrows,
                                                         int64_t nslots, int32_t C, int32_t b, const TX *G,
                                                         int64_t ldg, const TX *X, int64_t ldx, double alpha,
                                                         double *dsell) {
    for (int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < nslots;
         s += int64_t(gridDim.x) * blockDim.x) {
        if (s >= nrows) continue;
        const int64_t c = s / C, r = s - c * C;
        const int64_t row = perm ? int64_t(perm[s]) : s;
        const int len = cl[c];
        const int64_t base = cs[c] + r;
        const TX *g = G + row * ldg;
        for (int k = 0; k < len; ++k) {
            const int64_t e = base + int64_t(k) * C;
            const int ci = col[e];
            if (ci < 0) break;  // padding only follows the row's entries
            const TX *x = X + int64_t(ci) * ldx;
            double acc = 0.0;
            for (int j = 0; j < b; ++j) acc += double(g[j]) * double(x[j]);
            dsell[e] += alpha * acc;
        }
    }
}

// dval_csr[rowptr[i] + k] = dsell[entry k of row i] (or +=), one lane per row.
__global__ void __launch_bounds__(256) sell_to_csr_kernel(const double *dsell, const int64_t *rowptr,
                                                          const int32_t *rowslot, const int64_t *cs, int32_t C,
                                                          int64_t nrows, int accumulate, double *dval) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nrows;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t slot = rowslot[i];
        const int64_t c = slot / C, r = slot - c * C;
        const int64_t base = cs[c] + r;
        const int64_t p0 = rowptr[i], len = rowptr[i + 1] - p0;
        for (int64_t k = 0; k < len; ++k) {
            const double v = dsell[base + k * C];
            dval[p0 + k] = accumulate ? dval[p0 + k] + v : v;
        }
    }
}

// y = alpha x + beta y over n rows of b columns (row-major, leading dimension ld); y is not
// read when beta == 0.
template <class T>
__global__ void __launch_bounds__(256) axpby_kernel(int64_t n, int32_t b, int64_t ld, double alpha, const T *x,
                                                    double beta, T *y) {
    const int64_t N = n * b;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < N; e += int64_t(gridDim.x) * blockDim.x) {
        const int64_t i = e / b, k = i * ld + (e - i * b);
        const double v = alpha * double(x[k]);
        y[k] = T(beta != 0.0 ? v + beta * double(y[k]) : v);
    }
}

template <class V>
__global__ void __launch_bounds__(256) scatter_kernel(const double *src, const int64_t *pos, int64_t n, V *dst) {
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n; p += int64_t(gridDim.x) * blockDim.x)
        dst[pos[p]] = Conv<V, double>::go(src[p]);
}

static unsigned ggrid(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return unsigned(g);
}

int launch_grad_accum(const sell_mat *A, const void *G, int64_t ldg, const void *X, int64_t ldx, int vec_dt,
                      int32_t b, double alpha, double *dsell, hipStream_t s) {
    const HostSell &h = A->h;
    const int64_t nslots = h.nch * h.C;
    if (nslots == 0) return SELL_OK;
    if (vec_dt == SELL_F64)
        hipLaunchKernelGGL(grad_accum_kernel<double>, dim3(ggrid(nslots)), dim3(256), 0, s, A->d_col, A->d_cl,
                           A->d_cs, A->d_perm, h.nrows, nslots, h.C, b, static_cast<const double *>(G), ldg,
                           static_cast<const double *>(X), ldx, alpha, dsell);
    else
        hipLaunchKernelGGL(grad_accum_kernel<float>, dim3(ggrid(nslots)), dim3(256), 0, s, A->d_col, A->d_cl,
                           A->d_cs, A->d_perm, h.nrows, nslots, h.C, b, static_cast<const float *>(G), ldg,
                           static_cast<const float *>(X), ldx, alpha, dsell);
    return hipGetLastError() == hipSuccess ? SELL_OK : SELL_ERR_HIP;
}

int launch_sell_to_csr(const sell_mat *A, const double *dsell, int accumulate, double *dval, hipStream_t s) {
    const HostSell &h = A->h;
    if (h.nrows == 0) return SELL_OK;
    hipLaunchKernelGGL(sell_to_csr_kernel, dim3(ggrid(h.nrows)), dim3(256), 0, s, dsell, A->d_rowptr,
                       A->d_rowslot, A->d_cs, h.C, h.nrows, accumulate, dval);
    return hipGetLastError() == hipSuccess ? SELL_OK : SELL_ERR_HIP;
}

int launch_axpby(int vec_dt, int64_t n, int32_t b, int64_t ld, double alpha, const void *x, double beta, void *y,
                 hipStream_t s) {
    if (n * b == 0) return SELL_OK;
    if (vec_dt == SELL_F64)
        hipLaunchKernelGGL(axpby_kernel<double>, dim3(ggrid(n * b)), dim3(256), 0, s, n, b, ld, alpha,
                           static_cast<const double *>(x), beta, static_cast<double *>(y));
    else
        hipLaunchKernelGGL(axpby_kernel<float>, dim3(ggrid(n * b)), dim3(256), 0, s, n, b, ld, alpha,
                           static_cast<const float *>(x), beta, static_cast<float *>(y));
    return hipGetLastError() == hipSuccess ? SELL_OK : SELL_ERR_HIP;
}

int launch_scatter_values(const double *src, const int64_t *pos, int64_t n, int vdt, void *dst, hipStream_t s) {
    if (n == 0) return SELL_OK;
    if (vdt == SELL_F64)
        hipLaunchKernelGGL(scatter_kernel<double>, dim3(ggrid(n)), dim3(256), 0, s, src, pos, n,
                           static_cast<double *>(dst));
    else if (vdt == SELL_F32)
        hipLaunchKernelGGL(scatter_kernel<float>, dim3(ggrid(n)), dim3(256), 0, s, src, pos, n,
                           static_cast<float *>(dst));
    else
        hipLaunchKernelGGL(scatter_kernel<uint16_t>, dim3(ggrid(n)), dim3(256), 0, s, src, pos, n,
                           static_cast<uint16_t *>(dst));
    return hipGetLastError() == hipSuccess ? SELL_OK : SELL_ERR_HIP;
}

}  // namespace sellcs
