// spmmv_impl.h -- SELL-C-sigma sparse matrix times block vector kernels for gfx950.
//
// Operation (GHOST paper Sec. 5.1-5.3): for each row i and column j of a slice,
//     s_ij = sum_k A_ik X_kj                                   (plain product)
//     y_ij = alpha (s_ij - gamma_j x_ij) + beta y_ij            (augmented epilogue)
//     dots <y,y>_j, <x,y>_j, <x,x>_j of the final y;  z_ij = delta z_ij + eta y_ij.
//
// Mapping onto CDNA4 (wave64):
//   * One workgroup of kBlock threads owns one "tile": a contiguous range of chunks whose
//     cost (stored entries + row slots) is balanced at build time. Workgroup ids are
//     remapped so that each of the 8 XCDs (the hardware deals workgroups to XCDs in turn)
//     works on one contiguous eighth of the tiles; neighbouring rows then share an L2.
//   * Inside a tile, VL = B / VPT consecutive lanes serve one row slot, each lane owning
//     VPT consecutive columns of the row-major block vector, so a row of X is gathered by
//     VL lanes with contiguous addresses. Consecutive row slots of a chunk go to
//     consecutive lane groups, so the column-major chunk entries (value and index of
//     entry k of consecutive rows are adjacent) stream coalesced.
//   * The chunk loop is unrolled by 4 with all index/value loads issued before the
//     gathers, to keep enough loads in flight for HBM. Padding entries (column -1) are
//     skipped: no gather, no arithmetic.
//   * Dots are reduced without floating-point atomics: butterfly shuffles inside the
//     wave, LDS across the waves of the workgroup, one partial per tile in a workspace,
//     and the last workgroup to finish (an integer atomic ticket) sums the partials in
//     tile order. The order is fixed, so results are bitwise reproducible.
#pragma once

#include "internal.h"

namespace sellcs {

template <int VK>
struct KTypes;
template <>
struct KTypes<VK_F64F64> {
    using V = double;
    using X = double;
    using Acc = double;
};
template <>
struct KTypes<VK_F32F32> {
    using V = float;
    using X = float;
    using Acc = float;
};
template <>
struct KTypes<VK_BF16F32> {
    using V = uint16_t;
    using X = float;
    using Acc = float;
};

__device__ __forceinline__ double to_acc(double v, double) { return v; }
__device__ __forceinline__ float to_acc(float v, float) { return v; }
__device__ __forceinline__ float to_acc(uint16_t v, float) { return __uint_as_float(uint32_t(v) << 16); }

__device__ __forceinline__ double fmadd(double a, double b, double c) { return __fma_rn(a, b, c); }
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __fmaf_rn(a, b, c); }

// Workgroup id -> tile, so that XCD x (which receives workgroups x, x+8, x+16, ...)
// processes one contiguous range of tiles.
__device__ __forceinline__ int xcd_tile(int bid, int nblocks) {
    const int q = nblocks >> 3, r = nblocks & 7;
    const int x = bid & 7, k = bid >> 3;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

__device__ __forceinline__ double shfl_xor_d(double v, int m) { return __shfl_xor(v, m, 64); }

// Sum of the per-tile partials (laid out quantity-major: partials[q * ntiles + t]) by the
// last workgroup to finish; writes the requested dots.
__device__ __forceinline__ void finish_dots(const ProdArgs &a, int nq, int nb, int tile,
                                            const double *blocksum /* LDS, nq */) {
    __shared__ int s_last;
    const int tid = threadIdx.x;
    for (int q = tid; q < nq; q += kBlock) a.partials[size_t(q) * a.ntiles + tile] = blocksum[q];
    __threadfence();
    __syncthreads();
    if (tid == 0) s_last = (atomicAdd(a.counter, 1u) == unsigned(a.ntiles - 1));
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    const int lane = tid & 63, w = tid >> 6;
    for (int q = w; q < nq; q += kBlock / 64) {
        double s = 0.0;
        const double *p = a.partials + size_t(q) * a.ntiles;
        for (int t = lane; t < a.ntiles; t += 64) s += __builtin_nontemporal_load(p + t);
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) s += shfl_xor_d(s, m);
        if (lane == 0) {
            const int g = q / nb, j = q - g * nb;
            const uint32_t want = g == 0 ? SELL_SPMV_DOT_YY : g == 1 ? SELL_SPMV_DOT_XY : SELL_SPMV_DOT_XX;
            if (a.flags & want) a.dot[size_t(g) * a.dot_b + j] = s;
        }
    }
    if (tid == 0) *a.counter = 0u;
}

// B > 0: compile-time slice width with VPT columns per lane (VL = B / VPT lanes per row).
// B == 0: run-time width nb <= 64, one column per lane, VL = next power of two >= nb.
template <int VK, int B, int VPT, bool AUG>
__global__ void __launch_bounds__(kBlock) prod_kernel(ProdArgs a, int vl_log2) {
    using V = typename KTypes<VK>::V;
    using X = typename KTypes<VK>::X;
    using Acc = typename KTypes<VK>::Acc;
    constexpr bool DYN = (B == 0);
    const int nb = DYN ? a.nb : B;
    const int VL = DYN ? (1 << vl_log2) : (B / VPT);
    const int vls = DYN ? vl_log2 : __builtin_ctz(B / VPT);

    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int C = a.C;
    const int64_t s_begin = int64_t(a.tiles[tile]) * C;
    const int64_t s_end = int64_t(a.tiles[tile + 1]) * C;
    const int tid = threadIdx.x;
    const int vg = tid & (VL - 1);
    const int rows_per_pass = kBlock >> vls;
    const int jb = vg * VPT;
    const bool col_ok = DYN ? (vg < nb) : true;

    const V *__restrict__ val = static_cast<const V *>(a.val);
    const int32_t *__restrict__ col = a.col;
    const X *__restrict__ Xp = static_cast<const X *>(a.X);
    X *__restrict__ Yp = static_cast<X *>(a.Y);
    X *__restrict__ Zp = static_cast<X *>(a.Z);

    const bool want_dots = AUG && (a.flags & SELL_SPMV_DOTS);
    const bool shift = AUG && (a.flags & (SELL_SPMV_SHIFT | SELL_SPMV_VSHIFT));
    const bool need_x = shift || (AUG && (a.flags & (SELL_SPMV_DOT_XY | SELL_SPMV_DOT_XX)));
    const bool read_y = AUG && (a.flags & SELL_SPMV_AXPBY) && a.beta != 0.0;
    const bool chain = AUG && (a.flags & SELL_SPMV_CHAIN);
    const bool read_z = chain && a.delta != 0.0;
    const double alpha = (AUG && (a.flags & SELL_SPMV_SCALE)) ? a.alpha : 1.0;

    double dyy[VPT], dxy[VPT], dxx[VPT];
#pragma unroll
    for (int t = 0; t < VPT; ++t) dyy[t] = dxy[t] = dxx[t] = 0.0;

    for (int64_t s = s_begin + (tid >> vls); s < s_end; s += rows_per_pass) {
        const int64_t c = a.cshift >= 0 ? (s >> a.cshift) : int64_t(uint32_t(s) / uint32_t(C));
        const int r = int(s - c * C);
        const int len = a.cl[c];
        const int64_t base = a.cs[c] + r;
        Acc acc[VPT];
#pragma unroll
        for (int t = 0; t < VPT; ++t) acc[t] = Acc(0);

        if (col_ok) {
            int k = 0;
            for (; k + 4 <= len; k += 4) {
                int ci[4];
                V vv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    ci[u] = __builtin_nontemporal_load(col + base + int64_t(k + u) * C);
                    vv[u] = __builtin_nontemporal_load(val + base + int64_t(k + u) * C);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (ci[u] >= 0) {
                        const X *xr = Xp + int64_t(ci[u]) * a.xrs + int64_t(jb) * a.xcs;
                        const Acc v = to_acc(vv[u], Acc(0));
#pragma unroll
                        for (int t = 0; t < VPT; ++t) acc[t] = fmadd(v, Acc(xr[t * a.xcs]), acc[t]);
                    }
                }
            }
            for (; k < len; ++k) {
                const int ci = __builtin_nontemporal_load(col + base + int64_t(k) * C);
                const V vv = __builtin_nontemporal_load(val + base + int64_t(k) * C);
                if (ci >= 0) {
                    const X *xr = Xp + int64_t(ci) * a.xrs + int64_t(jb) * a.xcs;
                    const Acc v = to_acc(vv, Acc(0));
#pragma unroll
                    for (int t = 0; t < VPT; ++t) acc[t] = fmadd(v, Acc(xr[t * a.xcs]), acc[t]);
                }
            }
        }

        if (s < a.nrows && col_ok) {
            const int64_t row = a.perm ? int64_t(a.perm[s]) : s;
#pragma unroll
            for (int t = 0; t < VPT; ++t) {
                const int j = jb + t;
                X *yp = Yp + row * a.yrs + int64_t(j) * a.ycs;
                if (!AUG) {
                    *yp = X(acc[t]);
                } else {
                    double xv = 0.0;
                    if (need_x) xv = double(Xp[row * a.xrs + int64_t(j) * a.xcs]);
                    double tv = double(acc[t]);
                    if (shift) tv = tv - (a.has_gamma_v ? a.gamma_v[j] : a.gamma_s) * xv;
                    double y = alpha * tv;
                    if (read_y) y = y + a.beta * double(*yp);
                    const X ys = X(y);
                    *yp = ys;
                    const double yd = double(ys);
                    if (want_dots) {
                        dyy[t] += yd * yd;
                        dxy[t] += xv * yd;
                        dxx[t] += xv * xv;
                    }
                    if (chain) {
                        X *zp = Zp + row * a.zrs + int64_t(j) * a.zcs;
                        double z = a.eta * yd;
                        if (read_z) z = a.delta * double(*zp) + z;
                        *zp = X(z);
                    }
                }
            }
        }
    }

    if (!want_dots) return;

    // ---- deterministic dot reduction
    __shared__ double red[kBlock / 64][3 * kMaxSliceCols];
    __shared__ double bsum[3 * kMaxSliceCols];
    const int lane = tid & 63, w = tid >> 6;
#pragma unroll
    for (int t = 0; t < VPT; ++t) {
        for (int m = 32; m >= VL; m >>= 1) {
            dyy[t] += shfl_xor_d(dyy[t], m);
            dxy[t] += shfl_xor_d(dxy[t], m);
            dxx[t] += shfl_xor_d(dxx[t], m);
        }
    }
    if (lane < VL && col_ok) {
#pragma unroll
        for (int t = 0; t < VPT; ++t) {
            red[w][jb + t] = dyy[t];
            red[w][nb + jb + t] = dxy[t];
            red[w][2 * nb + jb + t] = dxx[t];
        }
    }
    __syncthreads();
    const int nq = 3 * nb;
    for (int q = tid; q < nq; q += kBlock) {
        double sum = 0.0;
#pragma unroll
        for (int ww = 0; ww < kBlock / 64; ++ww) sum += red[ww][q];
        bsum[q] = sum;
    }
    __syncthreads();
    finish_dots(a, nq, nb, tile, bsum);
}

// Transposed product by scattering with floating-point atomics: Y[col, j] += v * X[row, j].
template <int VK, int B, int VPT>
__global__ void __launch_bounds__(kBlock) transpose_kernel(ProdArgs a, int vl_log2) {
    using V = typename KTypes<VK>::V;
    using X = typename KTypes<VK>::X;
    using Acc = typename KTypes<VK>::Acc;
    constexpr bool DYN = (B == 0);
    const int nb = DYN ? a.nb : B;
    const int VL = DYN ? (1 << vl_log2) : (B / VPT);
    const int vls = DYN ? vl_log2 : __builtin_ctz(B / VPT);
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int C = a.C;
    const int64_t s_begin = int64_t(a.tiles[tile]) * C;
    const int64_t s_end = int64_t(a.tiles[tile + 1]) * C;
    const int tid = threadIdx.x;
    const int vg = tid & (VL - 1);
    const int jb = vg * VPT;
    if (DYN && vg >= nb) return;
    const V *__restrict__ val = static_cast<const V *>(a.val);
    const X *__restrict__ Xp = static_cast<const X *>(a.X);
    X *__restrict__ Yp = static_cast<X *>(a.Y);
    for (int64_t s = s_begin + (tid >> vls); s < s_end; s += (kBlock >> vls)) {
        if (s >= a.nrows) continue;
        const int64_t c = a.cshift >= 0 ? (s >> a.cshift) : int64_t(uint32_t(s) / uint32_t(C));
        const int r = int(s - c * C);
        const int len = a.cl[c];
        const int64_t base = a.cs[c] + r;
        const int64_t row = a.perm ? int64_t(a.perm[s]) : s;
        Acc xr[VPT];
#pragma unroll
        for (int t = 0; t < VPT; ++t) xr[t] = Acc(Xp[row * a.xrs + int64_t(jb + t) * a.xcs]);
        for (int k = 0; k < len; ++k) {
            const int ci = a.col[base + int64_t(k) * C];
            if (ci < 0) break;  // padding only follows the row's entries
            const Acc v = to_acc(val[base + int64_t(k) * C], Acc(0));
#pragma unroll
            for (int t = 0; t < VPT; ++t)
                unsafeAtomicAdd(Yp + int64_t(ci) * a.yrs + int64_t(jb + t) * a.ycs, X(v * xr[t]));
        }
    }
}

template <int VK, int B, int VPT, bool AUG>
inline int go_prod(const ProdArgs &a, hipStream_t s) {
    int vl_log2 = 0;
    if (B == 0) {
        while ((1 << vl_log2) < a.nb) ++vl_log2;
    }
    hipLaunchKernelGGL((prod_kernel<VK, B, VPT, AUG>), dim3(a.ntiles), dim3(kBlock), 0, s, a, vl_log2);
    return hipGetLastError() == hipSuccess ? SELL_OK : SELL_ERR_HIP;
}

template <int VK, int B, int VPT>
inline int go_transpose(const ProdArgs &a, hipStream_t s) {
    int vl_log2 = 0;
    if (B == 0) {
        while ((1 << vl_log2) < a.nb) ++vl_log2;
    }
    hipLaunchKernelGGL((transpose_kernel<VK, B, VPT>), dim3(a.ntiles), dim3(kBlock), 0, s, a, vl_log2);
    return hipGetLastError() == hipSuccess ? SELL_OK : SELL_ERR_HIP;
}

// Columns per lane for a compile-time width (tunable through SELLCS_VPT for experiments).
int choose_vpt(int vk, int b);

template <int VK, bool AUG>
int dispatch_prod(const ProdArgs &a, hipStream_t s, bool fixed_ok) {
    const int b = a.nb;
    const int vpt = choose_vpt(VK, b);
    if (fixed_ok) {
        switch (b) {
            case 1: return go_prod<VK, 1, 1, AUG>(a, s);
            case 2: return vpt >= 2 ? go_prod<VK, 2, 2, AUG>(a, s) : go_prod<VK, 2, 1, AUG>(a, s);
            case 4:
                return vpt >= 4 ? go_prod<VK, 4, 4, AUG>(a, s)
                                : vpt == 2 ? go_prod<VK, 4, 2, AUG>(a, s) : go_prod<VK, 4, 1, AUG>(a, s);
            case 8:
                return vpt >= 4 ? go_prod<VK, 8, 4, AUG>(a, s)
                                : vpt == 2 ? go_prod<VK, 8, 2, AUG>(a, s) : go_prod<VK, 8, 1, AUG>(a, s);
            case 16:
                return vpt >= 4 ? go_prod<VK, 16, 4, AUG>(a, s)
                                : vpt == 2 ? go_prod<VK, 16, 2, AUG>(a, s) : go_prod<VK, 16, 1, AUG>(a, s);
            case 32:
                return vpt >= 4 ? go_prod<VK, 32, 4, AUG>(a, s)
                                : vpt == 2 ? go_prod<VK, 32, 2, AUG>(a, s) : go_prod<VK, 32, 1, AUG>(a, s);
            default: break;
        }
    }
    return go_prod<VK, 0, 1, AUG>(a, s);
}

template <int VK>
int dispatch_transpose(const ProdArgs &a, hipStream_t s) {
    switch (a.nb) {
        case 1: return go_transpose<VK, 1, 1>(a, s);
        case 2: return go_transpose<VK, 2, 2>(a, s);
        case 4: return go_transpose<VK, 4, 4>(a, s);
        case 8: return go_transpose<VK, 8, 4>(a, s);
        case 16: return go_transpose<VK, 16, 4>(a, s);
        case 32: return go_transpose<VK, 32, 4>(a, s);
        default: return go_transpose<VK, 0, 1>(a, s);
    }
}

}  // namespace sellcs
