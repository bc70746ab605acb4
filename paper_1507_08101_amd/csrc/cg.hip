// cg.hip -- vector kernels of the conjugate-gradient drivers (block vectors, one CG per
// column, all scalars kept in FP64 on the device so an iteration needs no host sync).
//
// Column sums are deterministic: butterfly shuffles inside a wave, LDS across waves, one
// partial per workgroup (plain stores), then a one-workgroup-per-column kernel adds the
// partials in workgroup order and performs the per-column scalar updates.
#include <algorithm>
#include <initializer_list>
#include <type_traits>

#include "devutil.h"
#include "internal.h"

namespace sellcs {

constexpr int kVT = 256;  // threads per workgroup of the vector kernels

// Per-workgroup column sums of one FP64 value per thread (column j = tid & (bpad - 1);
// lanes with j >= b give 0), written with plain stores to partials[j * gridDim.x + block].
// Butterfly inside the wave, waves in order: a fixed order.
__device__ void colsum_store(double v, int bpad, int b, double *partials) {
    __shared__ double red[kVT / 64][64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int m = 32; m >= bpad; m >>= 1) v += __shfl_xor(v, m, 64);
    if (lane < bpad) red[w][lane] = v;
    __syncthreads();
    if (tid < b) {
        double s = 0.0;
#pragma unroll
        for (int ww = 0; ww < kVT / 64; ++ww) s += red[ww][tid];
        partials[size_t(tid) * gridDim.x + blockIdx.x] = s;
    }
}

// ---------------------------------------------------------------- 16-byte column groups
// The iteration's vector pass in the common case: b a multiple of the 16-byte group
// (4 floats or 2 doubles) with a power-of-two number of groups per row (TPR <= 16), rows 16-byte
// aligned. Each thread owns one group of every row it visits and keeps kVU (batched: kVUB) rows in
// flight, so a wave moves 1 KiB per load instruction. Every element is computed as in the
// per-element kernels (cg_rp_kernel and its batched form), which serve the other shapes; only the
// order in which the column sums are accumulated differs.
template <class T>
struct Vec16;
template <>
struct Vec16<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int V = 4;
};
template <>
struct Vec16<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int V = 2;
};

// rows in flight per thread of the single-system passes
constexpr int kVU = 4;
// the same for the batched pass, whose vectors span the whole batch: a sweep of 1 / 2 / 4 / 8 rows
// in flight over 1,024 to 8,192 workgroups, nontemporal or not, put 8 rows (nontemporal) first at
// every grid size (64 Laplacians at b = 8, 4,096 workgroups: BF16-value CG 0.681 s against 0.696
// with 4 rows, FP64 1.182 against 1.196 s)
constexpr int kVUB = 8;

template <bool NT, class VT>
__device__ __forceinline__ VT ld16(const VT *p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}
template <bool NT, class VT>
__device__ __forceinline__ void st16(VT v, VT *p) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Per-workgroup column sums when thread t holds the sums of columns (t % TPR) * V + v.
template <int V, int TPR>
__device__ void colsum_store_vec(const double (&acc)[V], double *partials) {
    __shared__ double red[kVT / 64][64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        double x = acc[v];
#pragma unroll
        for (int m = 32; m >= TPR; m >>= 1) x += __shfl_xor(x, m, 64);
        if (lane < TPR) red[w][lane * V + v] = x;
    }
    __syncthreads();
    if (tid < TPR * V) {
        double s = 0.0;
#pragma unroll
        for (int ww = 0; ww < kVT / 64; ++ww) s += red[ww][tid];
        partials[size_t(tid) * gridDim.x + blockIdx.x] = s;
    }
}

// Sum of n consecutive partials by one 256-thread workgroup (fixed order); thread 0 only.
__device__ double sum_partials(const double *p, int n) {
    double s = 0.0;
    for (int t = threadIdx.x; t < n; t += kVT) s += p[t];
    return block_sum_256(s);
}

// The scalars of iteration k for column j, from the product's tile partials of <q, q>
// (quantity j) and <p, q> (quantity b + j), q = A p:
//   alpha = rho / <p, q>,  beta = (alpha^2 <q, q> - rho) / rho.
// With r' = r - alpha q, <r', r'> = rho - 2 alpha <r, q> + alpha^2 <q, q>, and <r, q> = <p, q>
// because p - r is a multiple of the previous direction, which is A-conjugate to p; so the
// numerator of beta is <r', r'> before r' exists, and the residual, the step and the new
// direction are updated in one pass (the single-reduction form of Rupp et al., ACM TOMS 43(2),
// 2016). rho itself stays the directly summed <r, r>, which also decides convergence. A
// numerator that cancels to zero or below restarts the column from p = r' (beta = 0). After a
// reliable update keeps p but replaces r by the true residual, <r, q> = <p, q> holds only up to
// the drift that the update removed, and that iteration's beta carries the same small error.
__global__ void __launch_bounds__(kVT) cg_step_kernel(const double *prod_partials, int ntiles, int b, CgDev sc) {
    const int j = blockIdx.x;
    const double qq = sum_partials(prod_partials + size_t(j) * ntiles, ntiles);
    const double pq = sum_partials(prod_partials + size_t(b + j) * ntiles, ntiles);
    if (threadIdx.x == 0) {
        const double rho = sc.rho[j];
        const bool act = sc.active[j] != 0;
        const double al = (act && pq != 0.0) ? rho / pq : 0.0;
        const double num = al * al * qq - rho;
        sc.pq[j] = pq;
        sc.alpha[j] = al;
        sc.beta[j] = (act && rho != 0.0 && num > 0.0) ? num / rho : 0.0;
    }
}

// The iteration's vector pass: r' = r - alpha q, x += alpha p, p = r' + beta p, with the
// per-workgroup partials of <r', r'>. (x, the solution or the correction, takes the step
// along the direction before it is replaced.)
template <class T>
__global__ void __launch_bounds__(kVT) cg_rp_kernel(T *R, const T *Q, T *P, T *X, int64_t n, int b, int bpad,
                                                    int64_t ld, const double *alpha_v, const double *beta_v,
                                                    double *partials) {
    const int tid = threadIdx.x;
    const int j = tid & (bpad - 1);
    const int rows_per = kVT / bpad;
    double acc = 0.0;
    if (j < b) {
        const double al = alpha_v[j], be = beta_v[j];
        for (int64_t i = int64_t(blockIdx.x) * rows_per + tid / bpad; i < n; i += int64_t(gridDim.x) * rows_per) {
            const int64_t e = i * ld + j;
            const double p = double(P[e]);
            const T r = T(double(R[e]) - al * double(Q[e]));
            X[e] = T(double(X[e]) + al * p);
            P[e] = T(double(r) + be * p);
            R[e] = r;
            acc += double(r) * double(r);
        }
    }
    colsum_store(acc, bpad, b, partials);
}

// rho = <r, r> from the vector pass's partials; active &= rho > thresh2.
__global__ void __launch_bounds__(kVT) cg_rho_kernel(const double *partials, int G, CgDev sc) {
    const int j = blockIdx.x;
    const double rn = sum_partials(partials + size_t(j) * G, G);
    if (threadIdx.x == 0) {
        const bool act = sc.active[j] != 0;
        sc.rho[j] = rn;
        sc.active[j] = (act && rn > sc.thresh2[j]) ? 1 : 0;
    }
}

// cg_rp_kernel on 16-byte column groups (row pitch ldv groups)
template <class T, int TPR, int U = kVU, bool NT = false>
__global__ void __launch_bounds__(kVT) cg_rp_vec_kernel(T *R, const T *Q, T *P, T *X, int64_t n, int64_t ldv,
                                                        const double *alpha_v, const double *beta_v,
                                                        double *partials) {
    using VT = typename Vec16<T>::type;
    constexpr int V = Vec16<T>::V, rows_per = kVT / TPR;
    const int g = threadIdx.x % TPR;
    double al[V], be[V], acc[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        al[v] = alpha_v[g * V + v];
        be[v] = beta_v[g * V + v];
        acc[v] = 0.0;
    }
    VT *Rv = reinterpret_cast<VT *>(R);
    const VT *Qv = reinterpret_cast<const VT *>(Q);
    VT *Pv = reinterpret_cast<VT *>(P);
    VT *Xv = reinterpret_cast<VT *>(X);
    const int64_t st = int64_t(gridDim.x) * rows_per;
    for (int64_t i = int64_t(blockIdx.x) * rows_per + threadIdx.x / TPR; i < n; i += U * st) {
        VT rv[U] = {}, qv[U] = {}, pv[U] = {}, xv[U] = {};
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i + u * st < n) {
                const int64_t k = (i + u * st) * ldv + g;
                rv[u] = ld16<NT>(Rv + k);
                qv[u] = ld16<NT>(Qv + k);
                pv[u] = ld16<NT>(Pv + k);
                xv[u] = ld16<NT>(Xv + k);
            }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i + u * st < n) {
                VT ro, xo, po;
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const double p = double(pv[u][v]);
                    const T r = T(double(rv[u][v]) - al[v] * double(qv[u][v]));
                    ro[v] = r;
                    xo[v] = T(double(xv[u][v]) + al[v] * p);
                    po[v] = T(double(r) + be[v] * p);
                    acc[v] += double(r) * double(r);
                }
                const int64_t k = (i + u * st) * ldv + g;
                st16<NT>(ro, Rv + k);
                st16<NT>(xo, Xv + k);
                st16<NT>(po, Pv + k);
            }
    }
    colsum_store_vec<V, TPR>(acc, partials);
}

// per-workgroup partials of <U_j, V_j>
template <class T>
__global__ void __launch_bounds__(kVT) coldot_kernel(const T *U, const T *V, int64_t n, int b, int bpad,
                                                     int64_t ld, double *partials) {
    const int tid = threadIdx.x;
    const int j = tid & (bpad - 1);
    const int rows_per = kVT / bpad;
    double acc = 0.0;
    if (j < b)
        for (int64_t i = int64_t(blockIdx.x) * rows_per + tid / bpad; i < n; i += int64_t(gridDim.x) * rows_per)
            acc += double(U[i * ld + j]) * double(V[i * ld + j]);
    colsum_store(acc, bpad, b, partials);
}

// result_j = sum of the partials; optionally thresh2_j = f2 * (ref_j or result_j) and
// active_j = result_j > thresh2_j.
__global__ void __launch_bounds__(kVT) coldot_finish_kernel(const double *partials, int G, double *result,
                                                            double *thresh2, int32_t *active, const double *ref,
                                                            double f2) {
    const int j = blockIdx.x;
    const double v = sum_partials(partials + size_t(j) * G, G);
    if (threadIdx.x == 0) {
        result[j] = v;
        if (thresh2) {
            thresh2[j] = f2 * (ref ? ref[j] : v);
            active[j] = v > thresh2[j] ? 1 : 0;
        }
    }
}

// p = r in the columns with colmask[j] != 0 (one system)
template <class T>
__global__ void __launch_bounds__(kVT) copy_cols_kernel(T *P, const T *R, int64_t n, int b, int64_t ld,
                                                        const int32_t *colmask) {
    const int64_t N = n * b;
    for (int64_t e = int64_t(blockIdx.x) * kVT + threadIdx.x; e < N; e += int64_t(gridDim.x) * kVT) {
        const int64_t i = e / b;
        const int j = int(e - i * b);
        if (colmask[j]) P[i * ld + j] = R[i * ld + j];
    }
}

// x += d (the FP32 correction folded into the FP64 solution)
__global__ void __launch_bounds__(kVT) axpy_mixed_kernel(double *X, const float *D, int64_t n, int b, int64_t ld) {
    const int64_t N = n * b;
    for (int64_t e = int64_t(blockIdx.x) * kVT + threadIdx.x; e < N; e += int64_t(gridDim.x) * kVT) {
        const int64_t i = e / b;
        const int j = int(e - i * b);
        X[i * ld + j] += double(D[i * ld + j]);
    }
}

// ---------------------------------------------------------------- batched variants
// A batch of K independent systems stores its block vectors one after another (system m owns
// rows [row_off[m], row_off[m+1])). The workgroups of a vector launch are split over the
// systems: workgroups [vblk[m], vblk[m+1]) serve system m, so every workgroup works on one
// system and the per-system column sums stay deterministic. Workgroup partials go to
// partials[j * G + g] (G workgroups in total); those of system m, column j, are the
// contiguous range [j * G + vblk[m], j * G + vblk[m+1]). Scalars are indexed m * b + j.

__device__ __forceinline__ int seg_of(int g, const int32_t *blk, int K) {
    int lo = 0, hi = K;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (blk[mid] <= g)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Row loop of workgroup g over its system's rows: calls f(row) for the rows of this lane.
template <class F>
__device__ __forceinline__ void seg_rows(const BatchSeg &sg, int m, int bpad, F &&f) {
    const int g = blockIdx.x;
    const int lb = g - sg.vblk[m], nbl = sg.vblk[m + 1] - sg.vblk[m];
    const int rows_per = kVT / bpad;
    const int64_t r1 = sg.row_off[m + 1];
    for (int64_t i = sg.row_off[m] + int64_t(lb) * rows_per + threadIdx.x / bpad; i < r1;
         i += int64_t(nbl) * rows_per)
        f(i);
}

// alpha[m, j] and beta[m, j] of every system that iterates, as cg_step_kernel computes them, from
// the batched product's partials of matrix m (quantity t at pparts + 3 b pblk[m] + t npm,
// npm = pblk[m+1] - pblk[m]; <q, q> is quantity j, <p, q> quantity b + j). One workgroup per
// system and column (grid K x b).
__global__ void __launch_bounds__(kVT) bcg_step_kernel(const double *pparts, const int32_t *pblk, int b,
                                                       BatchCg sc) {
    const int m = blockIdx.x, j = blockIdx.y;
    if (!sc.sys_active[m]) return;
    const int npm = pblk[m + 1] - pblk[m];
    const double *base = pparts + size_t(3) * b * pblk[m];
    const double qq = sum_partials(base + size_t(j) * npm, npm);
    const double pq = sum_partials(base + size_t(b + j) * npm, npm);
    if (threadIdx.x == 0) {
        const int q = m * b + j;
        const double rho = sc.rho[q];
        const bool act = sc.active[q] != 0;
        const double al = (act && pq != 0.0) ? rho / pq : 0.0;
        const double num = al * al * qq - rho;
        sc.alpha[q] = al;
        sc.beta[q] = (act && rho != 0.0 && num > 0.0) ? num / rho : 0.0;
    }
}

// The vector pass of cg_rp_kernel on the rows of the systems that iterate: r' = r - alpha q,
// d += alpha p, p = r' + beta p, with the partials of <r', r'>.
template <class T>
__global__ void __launch_bounds__(kVT) bcg_rp_kernel(T *R, const T *Q, T *P, T *D, int b, int bpad, BatchSeg sg,
                                                     BatchCg sc, double *partials) {
    const int m = seg_of(blockIdx.x, sg.vblk, sg.K);
    const int j = threadIdx.x & (bpad - 1);
    double acc = 0.0;
    if (j < b && sc.sys_active[m]) {
        const double al = sc.alpha[m * b + j], be = sc.beta[m * b + j];
        seg_rows(sg, m, bpad, [&](int64_t i) {
            const int64_t e = i * b + j;
            const double p = double(P[e]);
            const T r = T(double(R[e]) - al * double(Q[e]));
            D[e] = T(double(D[e]) + al * p);
            P[e] = T(double(r) + be * p);
            R[e] = r;
            acc += double(r) * double(r);
        });
    }
    colsum_store(acc, bpad, b, partials);
}

// rho = <r, r> from the vector pass's partials; active &= rho > thresh2; the system stays
// active while one of its columns is; its iteration counter advances.
__global__ void __launch_bounds__(kVT) bcg_rho_kernel(const double *partials, int G, BatchSeg sg, int b,
                                                      BatchCg sc) {
    const int m = blockIdx.x;
    if (!sc.sys_active[m]) return;
    const int v0 = sg.vblk[m], nv = sg.vblk[m + 1] - v0;
    int any = 0;
    for (int j = 0; j < b; ++j) {
        const double rn = sum_partials(partials + size_t(j) * G + v0, nv);
        if (threadIdx.x == 0) {
            const int q = m * b + j;
            const int still = (sc.active[q] && rn > sc.thresh2[q]) ? 1 : 0;
            sc.rho[q] = rn;
            sc.active[q] = still;
            any |= still;
        }
    }
    if (threadIdx.x == 0) {
        sc.sys_active[m] = any;
        sc.iters[m] += 1;
    }
}

// bcg_rp_kernel on 16-byte column groups (b = TPR * V, rows contiguous)
template <class T, int TPR, int U = kVUB, bool NT = false>
__global__ void __launch_bounds__(kVT) bcg_rp_vec_kernel(T *R, const T *Q, T *P, T *D, BatchSeg sg, BatchCg sc,
                                                         double *partials) {
    using VT = typename Vec16<T>::type;
    constexpr int V = Vec16<T>::V, b = TPR * V, rows_per = kVT / TPR;
    const int m = seg_of(blockIdx.x, sg.vblk, sg.K);
    const int g = threadIdx.x % TPR;
    double acc[V];
#pragma unroll
    for (int v = 0; v < V; ++v) acc[v] = 0.0;
    if (sc.sys_active[m]) {
        double al[V], be[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            al[v] = sc.alpha[m * b + g * V + v];
            be[v] = sc.beta[m * b + g * V + v];
        }
        VT *Rv = reinterpret_cast<VT *>(R);
        const VT *Qv = reinterpret_cast<const VT *>(Q);
        VT *Pv = reinterpret_cast<VT *>(P);
        VT *Dv = reinterpret_cast<VT *>(D);
        const int lb = int(blockIdx.x) - sg.vblk[m], nbl = sg.vblk[m + 1] - sg.vblk[m];
        const int64_t r1 = sg.row_off[m + 1], st = int64_t(nbl) * rows_per;
        for (int64_t i = sg.row_off[m] + int64_t(lb) * rows_per + threadIdx.x / TPR; i < r1; i += U * st) {
            VT rv[U] = {}, qv[U] = {}, pv[U] = {}, dv[U] = {};
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (i + u * st < r1) {
                    const int64_t k = (i + u * st) * TPR + g;
                    rv[u] = ld16<NT>(Rv + k);
                    qv[u] = ld16<NT>(Qv + k);
                    pv[u] = ld16<NT>(Pv + k);
                    dv[u] = ld16<NT>(Dv + k);
                }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (i + u * st < r1) {
                    VT ro, dn, pn;
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const double p = double(pv[u][v]);
                        const T r = T(double(rv[u][v]) - al[v] * double(qv[u][v]));
                        ro[v] = r;
                        dn[v] = T(double(dv[u][v]) + al[v] * p);
                        pn[v] = T(double(r) + be[v] * p);
                        acc[v] += double(r) * double(r);
                    }
                    const int64_t k = (i + u * st) * TPR + g;
                    st16<NT>(ro, Rv + k);
                    st16<NT>(dn, Dv + k);
                    st16<NT>(pn, Pv + k);
                }
        }
    }
    colsum_store_vec<V, TPR>(acc, partials);
}

// Per-workgroup partials of <U_j, V_j> on the rows of the systems with mask[m] != 0
// (all systems when mask is null).
template <class T>
__global__ void __launch_bounds__(kVT) bcoldot_kernel(const T *U, const T *V, int b, int bpad, BatchSeg sg,
                                                      const int32_t *mask, double *partials) {
    const int m = seg_of(blockIdx.x, sg.vblk, sg.K);
    const int j = threadIdx.x & (bpad - 1);
    double acc = 0.0;
    if (j < b && (!mask || mask[m]))
        seg_rows(sg, m, bpad, [&](int64_t i) { acc += double(U[i * b + j]) * double(V[i * b + j]); });
    colsum_store(acc, bpad, b, partials);
}

// result[m, j] = sum of the partials of system m, column j (systems with mask[m] != 0 only);
// optionally thresh2[m, j] = f2 * (ref[m, j] or result[m, j]).
__global__ void __launch_bounds__(kVT) bcoldot_finish_kernel(const double *partials, int G, BatchSeg sg, int b,
                                                             const int32_t *mask, double *result, double *thresh2,
                                                             const double *ref, double f2) {
    const int m = blockIdx.x;
    if (mask && !mask[m]) return;
    const int v0 = sg.vblk[m], nv = sg.vblk[m + 1] - v0;
    for (int j = 0; j < b; ++j) {
        const double v = sum_partials(partials + size_t(j) * G + v0, nv);
        if (threadIdx.x == 0) {
            const int q = m * b + j;
            result[q] = v;
            if (thresh2) thresh2[q] = f2 * (ref ? ref[q] : v);
        }
    }
}

// Start of a residual refresh on the systems with mask[m] != 0: x += d, d = 0, r64 = b.
template <class T>
__global__ void __launch_bounds__(kVT) brefresh_prep_kernel(double *X, T *D, double *R64, const double *Bv, int b,
                                                            int bpad, BatchSeg sg, const int32_t *mask) {
    const int m = seg_of(blockIdx.x, sg.vblk, sg.K);
    const int j = threadIdx.x & (bpad - 1);
    if (j >= b || !mask[m]) return;
    seg_rows(sg, m, bpad, [&](int64_t i) {
        const int64_t e = i * b + j;
        X[e] += double(D[e]);
        D[e] = T(0);
        R64[e] = Bv[e];
    });
}

// r = T(r64) (round to nearest) on the systems with mask[m] != 0, with partials of <r, r>.
template <class T>
__global__ void __launch_bounds__(kVT) bconvert_kernel(T *R, const double *R64, int b, int bpad, BatchSeg sg,
                                                       const int32_t *mask, double *partials) {
    const int m = seg_of(blockIdx.x, sg.vblk, sg.K);
    const int j = threadIdx.x & (bpad - 1);
    double acc = 0.0;
    if (j < b && mask[m])
        seg_rows(sg, m, bpad, [&](int64_t i) {
            const T r = T(R64[i * b + j]);
            R[i * b + j] = r;
            acc += double(r) * double(r);
        });
    colsum_store(acc, bpad, b, partials);
}

// brefresh_prep_kernel and bconvert_kernel on groups of two columns (b even, b / 2 a power of
// two up to 16, rows 16-byte aligned): the FP64 rows move as 16-byte pieces, the rows of T as
// pairs, kVU rows in flight per thread. Every element is computed as in the per-element kernels.
template <class T>
struct Pair;
template <>
struct Pair<float> {
    typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct Pair<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};

template <class T, int TPR, int U, bool NT>
__global__ void __launch_bounds__(kVT) brefresh_prep_vec_kernel(double *X, T *D, double *R64, const double *Bv,
                                                                BatchSeg sg, const int32_t *mask) {
    using V2 = typename Pair<double>::type;
    using T2 = typename Pair<T>::type;
    constexpr int rows_per = kVT / TPR;
    const int m = seg_of(blockIdx.x, sg.vblk, sg.K);
    if (!mask[m]) return;
    const int g = threadIdx.x % TPR;
    V2 *Xv = reinterpret_cast<V2 *>(X);
    V2 *Rv = reinterpret_cast<V2 *>(R64);
    const V2 *Bvv = reinterpret_cast<const V2 *>(Bv);
    T2 *Dv = reinterpret_cast<T2 *>(D);
    const int lb = int(blockIdx.x) - sg.vblk[m], nbl = sg.vblk[m + 1] - sg.vblk[m];
    const int64_t r1 = sg.row_off[m + 1], st = int64_t(nbl) * rows_per;
    for (int64_t i = sg.row_off[m] + int64_t(lb) * rows_per + threadIdx.x / TPR; i < r1; i += U * st) {
        V2 xv[U] = {}, bv[U] = {};
        T2 dv[U] = {};
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i + u * st < r1) {
                const int64_t k = (i + u * st) * TPR + g;
                xv[u] = ld16<NT>(Xv + k);
                bv[u] = ld16<NT>(Bvv + k);
                dv[u] = ld16<NT>(Dv + k);
            }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i + u * st < r1) {
                const int64_t k = (i + u * st) * TPR + g;
                V2 xo;
                xo[0] = xv[u][0] + double(dv[u][0]);
                xo[1] = xv[u][1] + double(dv[u][1]);
                st16<NT>(xo, Xv + k);
                st16<NT>(T2{T(0), T(0)}, Dv + k);
                st16<NT>(bv[u], Rv + k);
            }
    }
}

template <class T, int TPR, int U, bool NT>
__global__ void __launch_bounds__(kVT) bconvert_vec_kernel(T *R, const double *R64, BatchSeg sg, const int32_t *mask,
                                                           double *partials) {
    using V2 = typename Pair<double>::type;
    using T2 = typename Pair<T>::type;
    constexpr int rows_per = kVT / TPR;
    const int m = seg_of(blockIdx.x, sg.vblk, sg.K);
    const int g = threadIdx.x % TPR;
    double acc[2] = {0.0, 0.0};
    if (mask[m]) {
        const V2 *Rs = reinterpret_cast<const V2 *>(R64);
        T2 *Rv = reinterpret_cast<T2 *>(R);
        const int lb = int(blockIdx.x) - sg.vblk[m], nbl = sg.vblk[m + 1] - sg.vblk[m];
        const int64_t r1 = sg.row_off[m + 1], st = int64_t(nbl) * rows_per;
        for (int64_t i = sg.row_off[m] + int64_t(lb) * rows_per + threadIdx.x / TPR; i < r1; i += U * st) {
            V2 sv[U] = {};
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (i + u * st < r1) sv[u] = ld16<NT>(Rs + (i + u * st) * TPR + g);
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (i + u * st < r1) {
                    T2 o;
                    o[0] = T(sv[u][0]);
                    o[1] = T(sv[u][1]);
                    acc[0] += double(o[0]) * double(o[0]);
                    acc[1] += double(o[1]) * double(o[1]);
                    st16<NT>(o, Rv + (i + u * st) * TPR + g);
                }
        }
    }
    colsum_store_vec<2, TPR>(acc, partials);
}

// p = r in the columns with colmask[m * b + j] != 0
template <class T>
__global__ void __launch_bounds__(kVT) bcopy_kernel(T *P, const T *R, int b, int bpad, BatchSeg sg,
                                                    const int32_t *colmask) {
    const int m = seg_of(blockIdx.x, sg.vblk, sg.K);
    const int j = threadIdx.x & (bpad - 1);
    if (j >= b || !colmask[m * b + j]) return;
    seg_rows(sg, m, bpad, [&](int64_t i) { P[i * b + j] = R[i * b + j]; });
}

// Dots of a batched product: dot[m * 3 nb + q] = sum of the partials of quantity q of matrix m
// (partials + 3 nb blk[m] + q npm, npm = blk[m+1] - blk[m]) for the requested groups.
__global__ void __launch_bounds__(kVT) batch_dot_finish_kernel(const double *partials, const int32_t *blk,
                                                               int32_t nb, uint32_t flags, double *dot) {
    const int q = blockIdx.x, m = blockIdx.y, g = q / nb;
    const uint32_t want = g == 0 ? SELL_SPMV_DOT_YY : g == 1 ? SELL_SPMV_DOT_XY : SELL_SPMV_DOT_XX;
    if (!(flags & want)) return;
    const int npm = blk[m + 1] - blk[m];
    const double v = sum_partials(partials + size_t(3) * nb * blk[m] + size_t(q) * npm, npm);
    if (threadIdx.x == 0) dot[size_t(m) * 3 * nb + q] = v;
}

// The same for a batch whose matrices have widths of their own (packed operands), per launch
// table position m: its partials start at 3 wmax blk[m] and hold 3 nbm[m] quantities (group g,
// column j at g * nbm[m] + j); its dots land packed at dot[3 dot_off[m] + g * nbm[m] + j].
__global__ void __launch_bounds__(kVT) batch_dot_finish_packed_kernel(const double *partials, const int32_t *blk,
                                                                      const int32_t *nbm, const int64_t *dot_off,
                                                                      int32_t wmax, uint32_t flags, double *dot) {
    const int q = blockIdx.x, m = blockIdx.y, g = q / wmax, j = q - g * wmax;
    const int w = nbm[m];
    if (j >= w) return;
    const uint32_t want = g == 0 ? SELL_SPMV_DOT_YY : g == 1 ? SELL_SPMV_DOT_XY : SELL_SPMV_DOT_XX;
    if (!(flags & want)) return;
    const int npm = blk[m + 1] - blk[m];
    const double v = sum_partials(partials + size_t(3) * wmax * blk[m] + size_t(g * w + j) * npm, npm);
    if (threadIdx.x == 0) dot[size_t(3) * dot_off[m] + size_t(g) * w + j] = v;
}

static unsigned vgrid(int64_t work, unsigned cap) {
    int64_t g = (work + kVT - 1) / kVT;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return unsigned(g);
}

static int pow2_at_least(int b) {
    int p = 1;
    while (p < b) p <<= 1;
    return p;
}

static int ok() { return hipGetLastError() == hipSuccess ? SELL_OK : SELL_ERR_HIP; }

unsigned cg_reduce_grid(int64_t n, int b) { return vgrid(n * pow2_at_least(b), kCgMaxGrid); }

int cg_launch_step(const double *prod_partials, int ntiles, int b, const CgDev &sc, hipStream_t s) {
    hipLaunchKernelGGL(cg_step_kernel, dim3(b), dim3(kVT), 0, s, prod_partials, ntiles, b, sc);
    return ok();
}

// Threads per row of the 16-byte-group kernels for b columns of T, row pitch ld, and the given
// pointers; 0 when those kernels do not apply.
template <class T>
static int group_tpr(int b, int64_t ld, std::initializer_list<const void *> ptrs) {
    constexpr int V = Vec16<T>::V;
    if (b < V || b % V || ld % V) return 0;
    const int tpr = b / V;
    if (tpr > 16 || (tpr & (tpr - 1))) return 0;
    for (const void *p : ptrs)
        if (reinterpret_cast<uintptr_t>(p) & 15u) return 0;
    return tpr;
}

// Calls f(std::integral_constant<int, TPR>) for tpr in {1, 2, 4, 8, 16}.
template <class F>
static void with_tpr(int tpr, F &&f) {
    switch (tpr) {
        case 1: f(std::integral_constant<int, 1>()); break;
        case 2: f(std::integral_constant<int, 2>()); break;
        case 4: f(std::integral_constant<int, 4>()); break;
        case 8: f(std::integral_constant<int, 8>()); break;
        default: f(std::integral_constant<int, 16>()); break;
    }
}

// Vectors of at least this many bytes are streamed past the caches (nontemporal loads and
// stores): with the iteration's four or five of them far larger than the 256 MB infinity cache
// nothing is reused from it, and the nontemporal path streams faster (batched FP64 CG of 64
// Laplacians, 710 MB vectors: 1.30 against 1.35 s). Smaller vectors stay cached: a 100^3 FP64
// CG with 64 MB vectors runs 72 ms nontemporal against 68 ms.
constexpr int64_t kNtBytes = int64_t(128) << 20;

// Calls f(std::bool_constant<nontemporal>) for vectors of n_elems elements of T.
template <class T, class F>
static void with_nt(int64_t n_elems, F &&f) {
    if (n_elems * int64_t(sizeof(T)) >= kNtBytes)
        f(std::true_type());
    else
        f(std::false_type());
}

static unsigned group_grid(int64_t n, int tpr, unsigned cap) {
    const int64_t rows_per = kVT / tpr;
    int64_t g = (n + rows_per * kVU - 1) / (rows_per * kVU);
    return unsigned(std::max<int64_t>(1, std::min<int64_t>(g, cap)));
}

template <class T>
static bool launch_rp_groups(T *R, const T *Q, T *P, T *X, int64_t n, int b, int64_t ld, const CgDev &sc,
                             double *partials, unsigned *grid, hipStream_t s) {
    const int tpr = group_tpr<T>(b, ld, {R, Q, P, X});
    if (!tpr) return false;
    const unsigned g = group_grid(n, tpr, kCgMaxGrid);
    with_tpr(tpr, [&](auto c) {
        constexpr int TPR = decltype(c)::value;
        with_nt<T>(n * ld, [&](auto nt) {
            hipLaunchKernelGGL((cg_rp_vec_kernel<T, TPR, kVU, decltype(nt)::value>), dim3(g), dim3(kVT), 0, s, R, Q, P,
                               X, n, ld / Vec16<T>::V, sc.alpha, sc.beta, partials);
        });
    });
    *grid = g;
    return true;
}

template <class T>
static void launch_rp(void *R, const void *Q, void *P, void *X, int64_t n, int b, int64_t ld, const CgDev &sc,
                      double *partials, unsigned *grid, hipStream_t s) {
    T *r = static_cast<T *>(R), *p = static_cast<T *>(P), *x = static_cast<T *>(X);
    const T *q = static_cast<const T *>(Q);
    if (n > 0 && launch_rp_groups(r, q, p, x, n, b, ld, sc, partials, grid, s)) return;
    *grid = cg_reduce_grid(n, b);
    hipLaunchKernelGGL(cg_rp_kernel<T>, dim3(*grid), dim3(kVT), 0, s, r, q, p, x, n, b, pow2_at_least(b), ld,
                       sc.alpha, sc.beta, partials);
}

int cg_launch_rp(int dt, void *R, const void *Q, void *P, void *X, int64_t n, int b, int64_t ld, const CgDev &sc,
                 double *partials, hipStream_t s) {
    unsigned g = 0;
    if (dt == SELL_F64)
        launch_rp<double>(R, Q, P, X, n, b, ld, sc, partials, &g, s);
    else
        launch_rp<float>(R, Q, P, X, n, b, ld, sc, partials, &g, s);
    if (ok() != SELL_OK) return SELL_ERR_HIP;
    hipLaunchKernelGGL(cg_rho_kernel, dim3(b), dim3(kVT), 0, s, partials, int(g), sc);
    return ok();
}

int cg_launch_coldot(int dt, const void *U, const void *V, int64_t n, int b, int64_t ld, double *result,
                     double *partials, double *thresh2, int32_t *active, const double *ref, double f2,
                     hipStream_t s) {
    const int bpad = pow2_at_least(b);
    const unsigned g = cg_reduce_grid(n, b);
    if (dt == SELL_F64)
        hipLaunchKernelGGL(coldot_kernel<double>, dim3(g), dim3(kVT), 0, s, static_cast<const double *>(U),
                           static_cast<const double *>(V), n, b, bpad, ld, partials);
    else
        hipLaunchKernelGGL(coldot_kernel<float>, dim3(g), dim3(kVT), 0, s, static_cast<const float *>(U),
                           static_cast<const float *>(V), n, b, bpad, ld, partials);
    if (ok() != SELL_OK) return SELL_ERR_HIP;
    hipLaunchKernelGGL(coldot_finish_kernel, dim3(b), dim3(kVT), 0, s, partials, int(g), result, thresh2, active,
                       ref, f2);
    return ok();
}

int cg_launch_copy_cols(int dt, void *P, const void *R, int64_t n, int b, int64_t ld, const int32_t *colmask,
                        hipStream_t s) {
    if (n * b == 0) return SELL_OK;
    if (dt == SELL_F64)
        hipLaunchKernelGGL(copy_cols_kernel<double>, dim3(vgrid(n * b, 4096)), dim3(kVT), 0, s,
                           static_cast<double *>(P), static_cast<const double *>(R), n, b, ld, colmask);
    else
        hipLaunchKernelGGL(copy_cols_kernel<float>, dim3(vgrid(n * b, 4096)), dim3(kVT), 0, s,
                           static_cast<float *>(P), static_cast<const float *>(R), n, b, ld, colmask);
    return ok();
}

int cg_launch_axpy_mixed(double *X, const float *D, int64_t n, int b, int64_t ld, hipStream_t s) {
    hipLaunchKernelGGL(axpy_mixed_kernel, dim3(vgrid(n * b, 4096)), dim3(kVT), 0, s, X, D, n, b, ld);
    return ok();
}

// ---------------------------------------------------------------- batched launchers
namespace {
template <class T>
T *tp(void *p) { return static_cast<T *>(p); }
template <class T>
const T *ctp(const void *p) { return static_cast<const T *>(p); }
}  // namespace

int bcg_launch_step(const double *pparts, const int32_t *pblk, int K, int b, const BatchCg &sc, hipStream_t s) {
    hipLaunchKernelGGL(bcg_step_kernel, dim3(K, b), dim3(kVT), 0, s, pparts, pblk, b, sc);
    return ok();
}

template <class T>
static void blaunch_rp(void *R, const void *Q, void *P, void *D, int b, const BatchSeg &sg, const BatchCg &sc,
                       double *partials, hipStream_t s) {
    T *r = tp<T>(R), *p = tp<T>(P), *d = tp<T>(D);
    const T *q = ctp<T>(Q);
    const int tpr = group_tpr<T>(b, b, {r, q, p, d});
    if (tpr) {
        with_tpr(tpr, [&](auto c) {
            constexpr int TPR = decltype(c)::value;
            with_nt<T>(sg.rows * b, [&](auto nt) {
                hipLaunchKernelGGL((bcg_rp_vec_kernel<T, TPR, kVUB, decltype(nt)::value>), dim3(sg.G), dim3(kVT), 0, s,
                                   r, q, p, d, sg, sc, partials);
            });
        });
        return;
    }
    hipLaunchKernelGGL(bcg_rp_kernel<T>, dim3(sg.G), dim3(kVT), 0, s, r, q, p, d, b, pow2_at_least(b), sg, sc,
                       partials);
}

int bcg_launch_rp(int dt, void *R, const void *Q, void *P, void *D, int b, const BatchSeg &sg, const BatchCg &sc,
                  double *partials, hipStream_t s) {
    if (dt == SELL_F64)
        blaunch_rp<double>(R, Q, P, D, b, sg, sc, partials, s);
    else
        blaunch_rp<float>(R, Q, P, D, b, sg, sc, partials, s);
    if (ok() != SELL_OK) return SELL_ERR_HIP;
    hipLaunchKernelGGL(bcg_rho_kernel, dim3(sg.K), dim3(kVT), 0, s, partials, sg.G, sg, b, sc);
    return ok();
}

int bcg_launch_coldot(int dt, const void *U, const void *V, int b, const BatchSeg &sg, const int32_t *mask,
                      double *partials, double *result, double *thresh2, const double *ref, double f2,
                      hipStream_t s) {
    const int bpad = pow2_at_least(b);
    if (dt == SELL_F64)
        hipLaunchKernelGGL(bcoldot_kernel<double>, dim3(sg.G), dim3(kVT), 0, s, ctp<double>(U), ctp<double>(V), b,
                           bpad, sg, mask, partials);
    else
        hipLaunchKernelGGL(bcoldot_kernel<float>, dim3(sg.G), dim3(kVT), 0, s, ctp<float>(U), ctp<float>(V), b,
                           bpad, sg, mask, partials);
    if (ok() != SELL_OK) return SELL_ERR_HIP;
    hipLaunchKernelGGL(bcoldot_finish_kernel, dim3(sg.K), dim3(kVT), 0, s, partials, sg.G, sg, b, mask, result,
                       thresh2, ref, f2);
    return ok();
}

// Groups of two columns per thread for b even with b / 2 a power of two up to 16 and the
// given pointers 16-byte aligned (0 otherwise).
static int pair_tpr(int b, std::initializer_list<const void *> ptrs) {
    if (b < 2 || b % 2) return 0;
    const int tpr = b / 2;
    if (tpr > 16 || (tpr & (tpr - 1))) return 0;
    for (const void *p : ptrs)
        if (reinterpret_cast<uintptr_t>(p) & 15u) return 0;
    return tpr;
}

template <class T>
static bool blaunch_prep_pairs(double *X, T *D, double *R64, const double *Bv, int b, const BatchSeg &sg,
                               const int32_t *mask, hipStream_t s) {
    const int tpr = pair_tpr(b, {X, D, R64, Bv});
    if (!tpr) return false;
    with_tpr(tpr, [&](auto c) {
        constexpr int TPR = decltype(c)::value;
        with_nt<double>(sg.rows * b, [&](auto nt) {
            hipLaunchKernelGGL((brefresh_prep_vec_kernel<T, TPR, kVU, decltype(nt)::value>), dim3(sg.G), dim3(kVT),
                               0, s, X, D, R64, Bv, sg, mask);
        });
    });
    return true;
}

template <class T>
static bool blaunch_convert_pairs(T *R, const double *R64, int b, const BatchSeg &sg, const int32_t *mask,
                                  double *partials, hipStream_t s) {
    const int tpr = pair_tpr(b, {R, R64});
    if (!tpr) return false;
    with_tpr(tpr, [&](auto c) {
        constexpr int TPR = decltype(c)::value;
        with_nt<double>(sg.rows * b, [&](auto nt) {
            hipLaunchKernelGGL((bconvert_vec_kernel<T, TPR, kVU, decltype(nt)::value>), dim3(sg.G), dim3(kVT), 0, s, R,
                               R64, sg, mask, partials);
        });
    });
    return true;
}

int bcg_launch_refresh_prep(int dt, double *X, void *D, double *R64, const double *Bv, int b, const BatchSeg &sg,
                            const int32_t *mask, hipStream_t s) {
    if (sg.G == 0) return SELL_OK;  // no workgroups: no system with rows to update
    if (dt == SELL_F64 ? blaunch_prep_pairs(X, tp<double>(D), R64, Bv, b, sg, mask, s)
                       : blaunch_prep_pairs(X, tp<float>(D), R64, Bv, b, sg, mask, s))
        return ok();
    const int bpad = pow2_at_least(b);
    if (dt == SELL_F64)
        hipLaunchKernelGGL(brefresh_prep_kernel<double>, dim3(sg.G), dim3(kVT), 0, s, X, tp<double>(D), R64, Bv, b,
                           bpad, sg, mask);
    else
        hipLaunchKernelGGL(brefresh_prep_kernel<float>, dim3(sg.G), dim3(kVT), 0, s, X, tp<float>(D), R64, Bv, b,
                           bpad, sg, mask);
    return ok();
}

int bcg_launch_convert(int dt, void *R, const double *R64, int b, const BatchSeg &sg, const int32_t *mask,
                       double *partials, double *rho, double *thresh2, const double *ref, double f2, hipStream_t s) {
    const int bpad = pow2_at_least(b);
    if (sg.G > 0 && !(dt == SELL_F64 ? blaunch_convert_pairs(tp<double>(R), R64, b, sg, mask, partials, s)
                                     : blaunch_convert_pairs(tp<float>(R), R64, b, sg, mask, partials, s))) {
        // (with no workgroups the finish below sums no partials: rho = 0)
        if (dt == SELL_F64)
            hipLaunchKernelGGL(bconvert_kernel<double>, dim3(sg.G), dim3(kVT), 0, s, tp<double>(R), R64, b, bpad, sg,
                               mask, partials);
        else
            hipLaunchKernelGGL(bconvert_kernel<float>, dim3(sg.G), dim3(kVT), 0, s, tp<float>(R), R64, b, bpad, sg,
                               mask, partials);
        if (ok() != SELL_OK) return SELL_ERR_HIP;
    }
    hipLaunchKernelGGL(bcoldot_finish_kernel, dim3(sg.K), dim3(kVT), 0, s, partials, sg.G, sg, b, mask, rho,
                       thresh2, ref, f2);
    return ok();
}

int bcg_launch_copy(int dt, void *P, const void *R, int b, const BatchSeg &sg, const int32_t *mask, hipStream_t s) {
    if (sg.G == 0) return SELL_OK;
    const int bpad = pow2_at_least(b);
    if (dt == SELL_F64)
        hipLaunchKernelGGL(bcopy_kernel<double>, dim3(sg.G), dim3(kVT), 0, s, tp<double>(P), ctp<double>(R), b, bpad,
                           sg, mask);
    else
        hipLaunchKernelGGL(bcopy_kernel<float>, dim3(sg.G), dim3(kVT), 0, s, tp<float>(P), ctp<float>(R), b, bpad,
                           sg, mask);
    return ok();
}

int launch_batch_dot_finish_packed(const double *partials, const int32_t *blk, const int32_t *nbm,
                                   const int64_t *dot_off, int K, int32_t wmax, uint32_t flags, double *dot,
                                   hipStream_t s) {
    if (K < 1) return SELL_OK;
    hipLaunchKernelGGL(batch_dot_finish_packed_kernel, dim3(3 * wmax, K), dim3(kVT), 0, s, partials, blk, nbm, dot_off,
                       wmax, flags, dot);
    return ok();
}

int launch_batch_dot_finish(const double *partials, const int32_t *blk, int K, int32_t nb, uint32_t flags,
                            double *dot, hipStream_t s) {
    if (K < 1) return SELL_OK;
    hipLaunchKernelGGL(batch_dot_finish_kernel, dim3(3 * nb, K), dim3(kVT), 0, s, partials, blk, nb, flags, dot);
    return ok();
}

}  // namespace sellcs
