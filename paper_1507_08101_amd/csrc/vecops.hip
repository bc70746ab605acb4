// vecops.hip -- block-vector kernels (fill, layout/type copy), value updates, KPM moment
// assembly, bandwidth probes, and the launch front-ends of the product kernels.
#include <cstdlib>
#include <map>
#include <utility>

#include "convert.h"
#include "devutil.h"
#include "internal.h"
#include "log.h"

namespace sellcs {

int prod_f64(ProdArgs &a, bool aug, bool fixed_ok, hipStream_t s);
int prod_f32(ProdArgs &a, bool aug, bool fixed_ok, hipStream_t s);
int prod_bf16(ProdArgs &a, bool aug, bool fixed_ok, hipStream_t s);
int transpose_f64(ProdArgs &a, hipStream_t s);
int transpose_f32(ProdArgs &a, hipStream_t s);
int transpose_bf16(ProdArgs &a, hipStream_t s);

// Columns per lane of the fixed-width kernels: up to four (16 bytes of a row per lane for
// FP32 vectors, two 16-byte pieces for FP64; measured fastest for FP64 at b = 8 on the
// 128^3 Anderson workload). SELLCS_VPT overrides the choice (1, 2 or 4) for tuning.
int choose_vpt(int vk, int b, int hint) {
    if ((hint == 1 || hint == 2 || hint == 4) && hint <= b) return hint;
    int v = b >= 4 ? 4 : b;
    if (const char *e = std::getenv("SELLCS_VPT")) {
        int x = std::atoi(e);
        if ((x == 1 || x == 2 || x == 4) && x <= b) v = x;
    }
    return v;
}

int32_t resident_grid(const void *kernel, int threads, int32_t ntiles, int32_t blocks_per_cu) {
    if (ntiles <= 0) return 0;
    // (workgroups per CU, CUs) of each kernel on each device
    static thread_local std::map<std::pair<int, const void *>, std::pair<int32_t, int32_t>> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    auto key = std::make_pair(dev, kernel);
    auto it = cache.find(key);
    std::pair<int32_t, int32_t> occ;
    if (it != cache.end()) {
        occ = it->second;
    } else {
        int per_cu = 0, ncu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
            per_cu = 1;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
            ncu = 256;
        if (const char *e = std::getenv("SELLCS_BLOCKS_PER_CU")) {
            const int v = std::atoi(e);
            if (v >= 1 && v <= 64) per_cu = v;
        }
        occ = std::make_pair(int32_t(per_cu), int32_t(ncu));
        cache.emplace(key, occ);
    }
    const int32_t per = (blocks_per_cu > 0 && blocks_per_cu < occ.first) ? blocks_per_cu : occ.first;
    const int64_t full = int64_t(per) * occ.second;
    return full < ntiles ? int32_t(full) : ntiles;
}

static bool fixed_width(int b) { return b == 1 || b == 2 || b == 4 || b == 8 || b == 16 || b == 32; }

static bool vec_ok(const void *p, int64_t rs, int64_t cs, int esize, int align) {
    return cs == 1 && (reinterpret_cast<uintptr_t>(p) % align) == 0 && ((rs * esize) % align) == 0;
}

int launch_product(ProdArgs &a, int vk, bool aug, hipStream_t s) {
    if (a.ntiles == 0) return SELL_OK;
    const int esize = vk == VK_F64F64 ? 8 : 4;
    const int vpt = choose_vpt(vk, a.nb, a.vpt_hint);
    const int align = vpt * esize < 16 ? vpt * esize : 16;
    bool fixed_ok = fixed_width(a.nb) && vec_ok(a.X, a.xrs, a.xcs, esize, align) &&
                    vec_ok(a.Y, a.yrs, a.ycs, esize, align);
    if (aug && (a.flags & SELL_SPMV_CHAIN)) fixed_ok = fixed_ok && vec_ok(a.Z, a.zrs, a.zcs, esize, align);
    if (!fixed_ok) {
        if (!fixed_width(a.nb))
            log_warn_once(kWarnProductWidth,
                          "block width %d has no fixed-width product kernel (1, 2, 4, 8, 16 and 32 have; "
                          "sell_set_slice splits a block into such slices): the run-time-width kernel runs",
                          a.nb);
        else
            log_warn_once(kWarnProductLayout,
                          "block vectors that are not row-major with %d-byte aligned rows (column-major, "
                          "strided or offset views): the run-time-width kernel runs",
                          align);
    }
    switch (vk) {
        case VK_F64F64: return prod_f64(a, aug, fixed_ok, s);
        case VK_F32F32: return prod_f32(a, aug, fixed_ok, s);
        case VK_BF16F32: return prod_bf16(a, aug, fixed_ok, s);
        default: return SELL_ERR_DTYPE;
    }
}

int launch_transpose_atomic(ProdArgs &a, int vk, hipStream_t s) {
    if (a.ntiles == 0) return SELL_OK;
    switch (vk) {
        case VK_F64F64: return transpose_f64(a, s);
        case VK_F32F32: return transpose_f32(a, s);
        case VK_BF16F32: return transpose_bf16(a, s);
        default: return SELL_ERR_DTYPE;
    }
}

static inline unsigned grid_for(int64_t n, int threads, unsigned cap = 8192) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return unsigned(g);
}

// ---------------------------------------------------------------- fill

template <class T>
__global__ void __launch_bounds__(256) fill_kernel(T *p, int64_t nrows, int32_t ncols, int64_t rs,
                                                   int64_t cs, T v) {
    const int64_t n = nrows * ncols;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
         e += int64_t(gridDim.x) * blockDim.x) {
        const int64_t i = e / ncols, j = e - i * ncols;
        p[i * rs + j * cs] = v;
    }
}

int launch_fill(void *p, int dt, int64_t nrows, int32_t ncols, int64_t rs, int64_t cs,
                double value, hipStream_t s) {
    const int64_t n = nrows * ncols;
    if (n == 0) return SELL_OK;
    const unsigned g = grid_for(n, 256);
    if (dt == SELL_F64)
        hipLaunchKernelGGL(fill_kernel<double>, dim3(g), dim3(256), 0, s, static_cast<double *>(p),
                           nrows, ncols, rs, cs, value);
    else if (dt == SELL_F32)
        hipLaunchKernelGGL(fill_kernel<float>, dim3(g), dim3(256), 0, s, static_cast<float *>(p), nrows,
                           ncols, rs, cs, float(value));
    else
        hipLaunchKernelGGL(fill_kernel<uint16_t>, dim3(g), dim3(256), 0, s,
                           static_cast<uint16_t *>(p), nrows, ncols, rs, cs, bf16_from_f64(value));
    return hipGetLastError() == hipSuccess ? SELL_OK : SELL_ERR_HIP;
}

// ---------------------------------------------------------------- block-vector copy

template <class D, class S>
__global__ void __launch_bounds__(256) copy_kernel(D *dst, int64_t drs, int64_t dcs, const S *src,
                                                   int64_t srs, int64_t scs, int64_t nrows,
                                                   int32_t ncols) {
    const int64_t n = nrows * ncols;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
         e += int64_t(gridDim.x) * blockDim.x) {
        // walk in destination order so the stores are contiguous
        int64_t i, j;
        if (dcs == 1) {
            i = e / ncols;
            j = e - i * ncols;
        } else {
            j = e / nrows;
            i = e - j * nrows;
        }
        dst[i * drs + j * dcs] = Conv<D, S>::go(src[i * srs + j * scs]);
    }
}

static void strides(const sell_bv *v, int64_t &rs, int64_t &cs) {
    if (v->lay == SELL_ROW_MAJOR) {
        rs = v->ld;
        cs = 1;
    } else {
        rs = 1;
        cs = v->ld;
    }
}

template <class D>
static int copy_from(const sell_bv *dst, const sell_bv *src, hipStream_t s) {
    int64_t drs, dcs, srs, scs;
    strides(dst, drs, dcs);
    strides(src, srs, scs);
    const unsigned g = grid_for(dst->nrows * dst->ncols, 256);
    D *d = static_cast<D *>(dst->ptr);
    if (src->dt == SELL_F64)
        hipLaunchKernelGGL((copy_kernel<D, double>), dim3(g), dim3(256), 0, s, d, drs, dcs,
                           static_cast<const double *>(src->ptr), srs, scs, dst->nrows, dst->ncols);
    else if (src->dt == SELL_F32)
        hipLaunchKernelGGL((copy_kernel<D, float>), dim3(g), dim3(256), 0, s, d, drs, dcs,
                           static_cast<const float *>(src->ptr), srs, scs, dst->nrows, dst->ncols);
    else
        hipLaunchKernelGGL((copy_kernel<D, uint16_t>), dim3(g), dim3(256), 0, s, d, drs, dcs,
                           static_cast<const uint16_t *>(src->ptr), srs, scs, dst->nrows, dst->ncols);
    return hipGetLastError() == hipSuccess ? SELL_OK : SELL_ERR_HIP;
}

int launch_copy(const sell_bv *dst, const sell_bv *src, hipStream_t s) {
    if (dst->nrows * dst->ncols == 0) return SELL_OK;
    if (dst->dt == SELL_F64) return copy_from<double>(dst, src, s);
    if (dst->dt == SELL_F32) return copy_from<float>(dst, src, s);
    return copy_from<uint16_t>(dst, src, s);
}

// ---------------------------------------------------------------- value update

template <class V>
__global__ void __launch_bounds__(256) update_values_kernel(V *sval, const double *csr_val,
                                                            const int64_t *rowptr,
                                                            const int32_t *rowslot,
                                                            const int64_t *cs, int32_t C,
                                                            int64_t nrows) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nrows;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t slot = rowslot[i];
        const int64_t c = slot / C, r = slot - c * C;
        const int64_t base = cs[c] + r;
        const int64_t p0 = rowptr[i], len = rowptr[i + 1] - p0;
        for (int64_t k = 0; k < len; ++k) sval[base + k * C] = Conv<V, double>::go(csr_val[p0 + k]);
    }
}

int launch_update_values(const sell_mat *A, const double *val_dev, hipStream_t s) {
    const int64_t n = A->h.nrows;
    if (n == 0) return SELL_OK;
    const unsigned g = grid_for(n, 256);
    if (A->h.vdt == SELL_F64)
        hipLaunchKernelGGL(update_values_kernel<double>, dim3(g), dim3(256), 0, s,
                           static_cast<double *>(A->d_val), val_dev, A->d_rowptr, A->d_rowslot, A->d_cs,
                           A->h.C, n);
    else if (A->h.vdt == SELL_F32)
        hipLaunchKernelGGL(update_values_kernel<float>, dim3(g), dim3(256), 0, s,
                           static_cast<float *>(A->d_val), val_dev, A->d_rowptr, A->d_rowslot, A->d_cs,
                           A->h.C, n);
    else
        hipLaunchKernelGGL(update_values_kernel<uint16_t>, dim3(g), dim3(256), 0, s,
                           static_cast<uint16_t *>(A->d_val), val_dev, A->d_rowptr, A->d_rowslot,
                           A->d_cs, A->h.C, n);
    return hipGetLastError() == hipSuccess ? SELL_OK : SELL_ERR_HIP;
}

// ---------------------------------------------------------------- dot partial sums

// blockIdx.x = quantity q = g * nb + j, blockIdx.y = batch entry k (its partials start at
// partials + k * part_stride).
__global__ void __launch_bounds__(256) dot_finish_kernel(const double *partials, int32_t nparts, int32_t nb,
                                                         uint32_t flags, double *dot, int32_t dot_b,
                                                         int64_t dot_stride, int64_t part_stride) {
    const int q = blockIdx.x, g = q / nb, j = q - g * nb;
    const uint32_t want = g == 0 ? SELL_SPMV_DOT_YY : g == 1 ? SELL_SPMV_DOT_XY : SELL_SPMV_DOT_XX;
    if (!(flags & want)) return;
    const double *p = partials + size_t(blockIdx.y) * size_t(part_stride) + size_t(q) * size_t(nparts);
    double s = 0.0;
    for (int t = threadIdx.x; t < nparts; t += 256) s += p[t];
    s = block_sum_256(s);
    if (threadIdx.x == 0) dot[size_t(blockIdx.y) * dot_stride + size_t(g) * dot_b + j] = s;
}

int launch_dot_finish(const double *partials, int32_t nparts, int32_t nb, uint32_t flags, double *dot,
                      int32_t dot_b, int64_t batch, int64_t dot_stride, hipStream_t s) {
    return launch_dot_finish_strided(partials, nparts, nb, flags, dot, dot_b, batch, dot_stride,
                                     int64_t(3) * nb * nparts, s);
}

int launch_dot_finish_strided(const double *partials, int32_t nparts, int32_t nb, uint32_t flags, double *dot,
                              int32_t dot_b, int64_t batch, int64_t dot_stride, int64_t part_stride,
                              hipStream_t s) {
    if (batch < 1 || nparts < 1) return SELL_OK;
    hipLaunchKernelGGL(dot_finish_kernel, dim3(3 * nb, unsigned(batch)), dim3(256), 0, s, partials, nparts, nb,
                       flags, dot, dot_b, dot_stride, part_stride);
    return hipGetLastError() == hipSuccess ? SELL_OK : SELL_ERR_HIP;
}

// ---------------------------------------------------------------- KPM moments
// dots: M groups of 3b doubles [<y,y> | <x,y> | <x,x>] written by the M augmented products
// of the recurrence; step 0 has x = v0, y = v1; step m >= 1 has x = v_m, y = v_{m+1}.
// Chebyshev doubling: T_2m = 2 T_m^2 - T_0 and T_2m+1 = 2 T_m T_m+1 - T_1, so for a
// symmetric matrix mu_2m = 2 <v_m, v_m> - mu_0 and mu_2m+1 = 2 <v_m+1, v_m> - mu_1.
__global__ void kpm_moments_kernel(const double *dots, int64_t M, int32_t b, double *mu) {
    const int64_t g = 3 * int64_t(b);
    const int64_t total = (2 * M + 1) * int64_t(b);
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
         e += int64_t(gridDim.x) * blockDim.x) {
        const int64_t k = e / b;
        const int j = int(e - k * b);
        const double mu0 = dots[2 * b + j];  // <v0, v0>
        const double mu1 = dots[b + j];      // <v0, v1>
        double r;
        if (k == 0)
            r = mu0;
        else if (k == 1)
            r = mu1;
        else if (k % 2 == 0)
            r = 2.0 * dots[(k / 2 - 1) * g + j] - mu0;  // 2 <v_m, v_m> - mu0, m = k/2
        else
            r = 2.0 * dots[((k - 1) / 2) * g + b + j] - mu1;  // 2 <v_m, v_m+1> - mu1, m = (k-1)/2
        mu[e] = r;
    }
}

int launch_kpm_moments(const double *dots, int64_t M, int32_t b, double *mu, hipStream_t s) {
    const unsigned g = grid_for((2 * M + 1) * b, 256, 1024);
    hipLaunchKernelGGL(kpm_moments_kernel, dim3(g), dim3(256), 0, s, dots, M, b, mu);
    return hipGetLastError() == hipSuccess ? SELL_OK : SELL_ERR_HIP;
}

// ---------------------------------------------------------------- bandwidth probes
// Plain streaming kernels over 16-byte elements, 4 loads in flight per thread, nontemporal
// hints so the probe measures HBM and not the caches.

typedef float f4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) probe_copy(f4 *__restrict__ d, const f4 *__restrict__ s, int64_t n) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        f4 a = __builtin_nontemporal_load(s + i), b = __builtin_nontemporal_load(s + i + stride);
        f4 c = __builtin_nontemporal_load(s + i + 2 * stride), e = __builtin_nontemporal_load(s + i + 3 * stride);
        __builtin_nontemporal_store(a, d + i);
        __builtin_nontemporal_store(b, d + i + stride);
        __builtin_nontemporal_store(c, d + i + 2 * stride);
        __builtin_nontemporal_store(e, d + i + 3 * stride);
    }
    for (; i < n; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(s + i), d + i);
}

__global__ void __launch_bounds__(256) probe_read(float *__restrict__ d, const f4 *__restrict__ s, int64_t n) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    for (; i + 3 * stride < n; i += 4 * stride) {
        f4 a = __builtin_nontemporal_load(s + i), b = __builtin_nontemporal_load(s + i + stride);
        f4 c = __builtin_nontemporal_load(s + i + 2 * stride), e = __builtin_nontemporal_load(s + i + 3 * stride);
        acc += (a + b) + (c + e);
    }
    for (; i < n; i += stride) acc += __builtin_nontemporal_load(s + i);
    const float t = acc.x + acc.y + acc.z + acc.w;
    if (t == 1.2345e-30f) d[threadIdx.x] = t;  // keeps the loads alive; practically never taken
}

__global__ void __launch_bounds__(256) probe_write(f4 *__restrict__ d, int64_t n) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    const f4 v = {1.f, 2.f, 3.f, 4.f};
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        __builtin_nontemporal_store(v, d + i);
}

// The same copy and write with ordinary (cached) loads and stores.
__global__ void __launch_bounds__(256) probe_copy_plain(f4 *__restrict__ d, const f4 *__restrict__ s, int64_t n) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const f4 a = s[i], b = s[i + stride], c = s[i + 2 * stride], e = s[i + 3 * stride];
        d[i] = a;
        d[i + stride] = b;
        d[i + 2 * stride] = c;
        d[i + 3 * stride] = e;
    }
    for (; i < n; i += stride) d[i] = s[i];
}

__global__ void __launch_bounds__(256) probe_write_plain(f4 *__restrict__ d, int64_t n) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    const f4 v = {1.f, 2.f, 3.f, 4.f};
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) d[i] = v;
}

// Streams of R reads and W (0 or 1) writes over 16-byte elements: element i of the write
// stream is the sum of element i of the R read streams (stream r at src + r n); with W = 0 the
// sums are reduced to one 16-byte partial per workgroup in sink. U elements per stream and
// thread in flight per iteration (R U loads), grid-stride over the arrays.
template <bool NT>
__device__ __forceinline__ f4 probe_ld(const f4 *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <bool NT>
__device__ __forceinline__ void probe_st(f4 v, f4 *p) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <int R, int W, int U, bool NT>
__global__ void __launch_bounds__(256) probe_stream_kernel(f4 *__restrict__ d, const f4 *__restrict__ s, int64_t n,
                                                           f4 *__restrict__ sink) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const f4 one = {1.f, 2.f, 3.f, 4.f};
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    for (; i + (U - 1) * stride < n; i += U * stride) {
        f4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = R == 0 ? one : f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] += probe_ld<NT>(s + r * n + i + u * stride);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if constexpr (W == 1) probe_st<NT>(v[u], d + i + u * stride);
            else acc += v[u];
        }
    }
    for (; i < n; i += stride) {
        f4 v = R == 0 ? one : f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < R; ++r) v += probe_ld<NT>(s + r * n + i);
        if constexpr (W == 1) probe_st<NT>(v, d + i);
        else acc += v;
    }
    if constexpr (W == 0) {
        __shared__ f4 part[256];
        part[threadIdx.x] = acc;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (int(threadIdx.x) < h) part[threadIdx.x] += part[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) sink[blockIdx.x] = part[0];
    }
}

template <int R, int W, int U>
void launch_stream_u(bool nt, unsigned g, f4 *d, const f4 *sp, int64_t n, hipStream_t s) {
    if (nt) hipLaunchKernelGGL((probe_stream_kernel<R, W, U, true>), dim3(g), dim3(256), 0, s, d, sp, n, d);
    else hipLaunchKernelGGL((probe_stream_kernel<R, W, U, false>), dim3(g), dim3(256), 0, s, d, sp, n, d);
}

template <int R, int W>
void launch_stream_rw(int unroll, bool nt, unsigned g, f4 *d, const f4 *sp, int64_t n, hipStream_t s) {
    switch (unroll) {
        case 1: launch_stream_u<R, W, 1>(nt, g, d, sp, n, s); break;
        case 2: launch_stream_u<R, W, 2>(nt, g, d, sp, n, s); break;
        case 4: launch_stream_u<R, W, 4>(nt, g, d, sp, n, s); break;
        default: launch_stream_u<R, W, 8>(nt, g, d, sp, n, s); break;
    }
}

int launch_probe_stream(int reads, int writes, int unroll, int nontemporal, int grid, void *dst, const void *src,
                        int64_t bytes, hipStream_t s) {
    const int64_t n = bytes / 16;
    f4 *d = static_cast<f4 *>(dst);
    const f4 *sp = static_cast<const f4 *>(src);
    const unsigned g = unsigned(grid);
    const bool nt = nontemporal != 0;
    const int key = reads * 2 + writes;
    switch (key) {
        case 1: launch_stream_rw<0, 1>(unroll, nt, g, d, sp, n, s); break;
        case 2: launch_stream_rw<1, 0>(unroll, nt, g, d, sp, n, s); break;
        case 3: launch_stream_rw<1, 1>(unroll, nt, g, d, sp, n, s); break;
        case 4: launch_stream_rw<2, 0>(unroll, nt, g, d, sp, n, s); break;
        case 5: launch_stream_rw<2, 1>(unroll, nt, g, d, sp, n, s); break;
        case 6: launch_stream_rw<3, 0>(unroll, nt, g, d, sp, n, s); break;
        case 7: launch_stream_rw<3, 1>(unroll, nt, g, d, sp, n, s); break;
        case 8: launch_stream_rw<4, 0>(unroll, nt, g, d, sp, n, s); break;
        case 9: launch_stream_rw<4, 1>(unroll, nt, g, d, sp, n, s); break;
        default: return SELL_ERR_ARG;
    }
    return hipGetLastError() == hipSuccess ? SELL_OK : SELL_ERR_HIP;
}

int launch_probe(int kind, void *dst, const void *src, int64_t bytes, hipStream_t s) {
    const int64_t n = bytes / 16;
    const unsigned g = 256 * 16;
    f4 *d = static_cast<f4 *>(dst);
    const f4 *sp = static_cast<const f4 *>(src);
    switch (kind) {
        case 0: hipLaunchKernelGGL(probe_copy, dim3(g), dim3(256), 0, s, d, sp, n); break;
        case 1: hipLaunchKernelGGL(probe_read, dim3(g), dim3(256), 0, s, static_cast<float *>(dst), sp, n); break;
        case 2: hipLaunchKernelGGL(probe_write, dim3(g), dim3(256), 0, s, d, n); break;
        case 3: hipLaunchKernelGGL(probe_copy_plain, dim3(g), dim3(256), 0, s, d, sp, n); break;
        default: hipLaunchKernelGGL(probe_write_plain, dim3(g), dim3(256), 0, s, d, n); break;
    }
    return hipGetLastError() == hipSuccess ? SELL_OK : SELL_ERR_HIP;
}

}  // namespace sellcs
