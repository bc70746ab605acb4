// kpm_dos.hip -- density of states from block KPM moments (the kernel polynomial method that
// the fused block product serves; the reconstruction is the textbook one: block-averaged
// normalised moments, Jackson damping, Chebyshev series over the weight 1/(pi sqrt(1-x^2))).
#include <cmath>

#include "internal.h"

namespace sellcs {

namespace {

constexpr int kDT = 256;       // energies per workgroup
constexpr int kChunk = 2048;   // damped moments staged in LDS at a time

// One thread per energy. The workgroup stages d_m = (m ? 2 : 1) g_m sum_j mu[m, j] / sum_j mu[0, j]
// in LDS, a chunk of moments at a time; every thread carries T_{m-1}(x), T_m(x) across chunks
// (three-term recurrence) and accumulates sum_m d_m T_m(x).
__global__ void __launch_bounds__(kDT) kpm_dos_kernel(const double *__restrict__ mu, int64_t nmom, int b,
                                                      int jackson, double s, double c, const double *__restrict__ E,
                                                      int64_t K, double *__restrict__ rho) {
    __shared__ double d[kChunk];
    __shared__ double inv0;
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int j = 0; j < b; ++j) t += mu[j];
        inv0 = 1.0 / t;
    }
    const int64_t k = int64_t(blockIdx.x) * kDT + threadIdx.x;
    const double x = k < K ? (E[k] - c) / s : 0.0;
    const double q = M_PI / double(nmom + 1);
    const double cotq = cos(q) / sin(q);
    double tprev = x, tcur = 1.0, acc = 0.0;  // T_{-1} := T_1 makes the recurrence give T_1 = x
    __syncthreads();
    for (int64_t base = 0; base < nmom; base += kChunk) {
        const int cnt = nmom - base < kChunk ? int(nmom - base) : kChunk;
        for (int e = threadIdx.x; e < cnt; e += kDT) {
            const int64_t m = base + e;
            double sm = 0.0;
            for (int j = 0; j < b; ++j) sm += mu[m * b + j];
            const double g =
                jackson ? (double(nmom - m + 1) * cos(q * double(m)) + sin(q * double(m)) * cotq) / double(nmom + 1)
                        : 1.0;
            d[e] = (m == 0 ? 1.0 : 2.0) * g * sm * inv0;
        }
        __syncthreads();
        for (int e = 0; e < cnt; ++e) {
            acc = fma(d[e], tcur, acc);
            const double tn = 2.0 * x * tcur - tprev;
            tprev = tcur;
            tcur = tn;
        }
        __syncthreads();
    }
    if (k < K) rho[k] = fabs(x) < 1.0 ? acc / (M_PI * sqrt(1.0 - x * x) * s) : 0.0;
}

}  // namespace

}  // namespace sellcs

using namespace sellcs;

extern "C" int sell_kpm_dos(const double *mu, int64_t nmom, int32_t b, int32_t kernel, double s, double c,
                            const double *E, int64_t K, double *rho, void *stream) {
    if (nmom < 1 || b < 1 || K < 0 || !mu) return SELL_ERR_ARG;
    if (kernel != SELL_KPM_NONE && kernel != SELL_KPM_JACKSON) return SELL_ERR_ARG;
    if (!(s > 0.0) || !std::isfinite(s) || !std::isfinite(c)) return SELL_ERR_ARG;
    if (K > 0 && (!E || !rho)) return SELL_ERR_ARG;
    if (K == 0) return SELL_OK;
    const int64_t g = (K + kDT - 1) / kDT;
    if (g > int64_t(0x7fffffff)) return SELL_ERR_ARG;
    hipLaunchKernelGGL(kpm_dos_kernel, dim3(unsigned(g)), dim3(kDT), 0, static_cast<hipStream_t>(stream), mu, nmom,
                       int(b), kernel == SELL_KPM_JACKSON ? 1 : 0, s, c, E, K, rho);
    return hipGetLastError() == hipSuccess ? SELL_OK : SELL_ERR_HIP;
}
