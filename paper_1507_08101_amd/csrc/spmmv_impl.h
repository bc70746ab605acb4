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
//   * The chunk loop takes batches of U entries (8, or 7 and 5 for rows of that length),
//     issuing all index/value loads of a batch before its gathers, to keep enough loads in
//     flight. Batch slots past the chunk length are clamped to its last entry and skipped in
//     the arithmetic; padding entries inside it (value 0 and the row's last real column) are
//     gathered and multiplied like the others, which keeps the loop free of branches.
//   * What bounds the kernel is the bytes its gathers carry through each CU's vector memory
//     path (texture address and data units), more than HBM or where the gathers hit. So lanes
//     that gather 32 bytes per entry run one workgroup per CU by default, and the KPM step's
//     compile-time copy takes the diagonal entry from the row's own x (already loaded for the
//     shift and the dots), with that lane masked off the gather.
//   * Optionally (STG) x is gathered from a cache of x pages in LDS, filled by asynchronous
//     global-to-LDS copies of the next work unit's pages during the current one, with
//     16-bit unit-local column indices (stage.hip builds them and the slot plan).
//   * Dots are reduced without floating-point atomics: butterfly shuffles inside the
//     wave, LDS across the waves of the workgroup, one partial per tile written with a
//     plain store; a separate small kernel (or the caller's next kernel) sums the partials
//     in tile order. The order is fixed, so results are bitwise reproducible. There is no
//     "last workgroup" ticket: on a multi-XCD part the device-scope release/acquire it
//     needs writes back and invalidates the L2 once per workgroup.
#pragma once

#include <algorithm>
#include <type_traits>

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

// Pointers into global memory. Pointers read from memory (the argument tables of the batched
// kernel) are generic to the compiler, which would access them with flat instructions (that
// also count against the LDS counter and so lengthen every wait); typed as global pointers
// they are accessed with global loads and stores, as pointers passed as kernel arguments are.
#define SELL_GLOBAL __attribute__((address_space(1)))

template <class T>
__device__ __forceinline__ SELL_GLOBAL T *to_global(T *p) {
    return (SELL_GLOBAL T *)p;
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// VPT consecutive elements at p (element stride cs). VEC: cs == 1 and p aligned to
// min(16, VPT * sizeof(X)) bytes, so the row piece moves as 8- or 16-byte vector accesses.
template <class X, int VPT, bool VEC>
__device__ __forceinline__ void load_row(const SELL_GLOBAL X *p, int64_t cs, X (&o)[VPT]) {
    constexpr int bytes = VPT * int(sizeof(X));
    if constexpr (VEC && bytes % 16 == 0) {
#pragma unroll
        for (int q = 0; q < bytes / 16; ++q) {
            const u32x4 v = reinterpret_cast<const SELL_GLOBAL u32x4 *>(p)[q];
            __builtin_memcpy(reinterpret_cast<char *>(o) + 16 * q, &v, 16);
        }
    } else if constexpr (VEC && bytes == 8) {
        const u32x2 v = *reinterpret_cast<const SELL_GLOBAL u32x2 *>(p);
        __builtin_memcpy(o, &v, 8);
    } else {
#pragma unroll
        for (int t = 0; t < VPT; ++t) o[t] = p[t * cs];
    }
}

// Row stores are nontemporal: the product never reads its outputs again in the same launch.
template <class X, int VPT, bool VEC>
__device__ __forceinline__ void store_row(SELL_GLOBAL X *p, int64_t cs, const X (&o)[VPT]) {
    constexpr int bytes = VPT * int(sizeof(X));
    if constexpr (VEC && bytes % 16 == 0) {
#pragma unroll
        for (int q = 0; q < bytes / 16; ++q) {
            u32x4 v;
            __builtin_memcpy(&v, reinterpret_cast<const char *>(o) + 16 * q, 16);
            __builtin_nontemporal_store(v, reinterpret_cast<SELL_GLOBAL u32x4 *>(p) + q);
        }
    } else if constexpr (VEC && bytes == 8) {
        u32x2 v;
        __builtin_memcpy(&v, o, 8);
        __builtin_nontemporal_store(v, reinterpret_cast<SELL_GLOBAL u32x2 *>(p));
    } else {
#pragma unroll
        for (int t = 0; t < VPT; ++t) p[t * cs] = o[t];
    }
}

// Entries gathered per batch: all index/value loads of a batch are issued before its
// gathers, and all gathers before the FMAs, so a row of up to U entries costs one round of
// index loads and one round of gathers. The default is 8; the fixed-width kernels also come
// with 7 and 5 (rows of 7 and 5 entries). The gathered values take U * VPT * sizeof(X) / 4
// VGPRs (at most 64 with 4 FP64 columns per lane).
constexpr int kBatchDefault = 8;

// B > 0: compile-time slice width with VPT columns per lane (VL = B / VPT lanes per row);
//        the block vectors are row-major with rows aligned for vector accesses (VEC).
// B == 0: run-time width nb <= 64, one column per lane, VL = next power of two >= nb,
//         any strides.
// The product over the tiles of workgroup `tile` (one of a.nblocks) of one matrix.
// FL != 0: the augmentation flags are known at compile time (a.flags == FL), so the unused
// parts of the epilogue take no registers.
template <int VK, int B, int VPT, bool AUG, int UB = 0, bool STG = false, uint32_t FL = 0>
__device__ __forceinline__ void prod_body(const ProdArgs &a, const int tile, const int vl_log2) {
    using V = typename KTypes<VK>::V;
    using X = typename KTypes<VK>::X;
    using Acc = typename KTypes<VK>::Acc;
    constexpr bool DYN = (B == 0);
    constexpr bool VEC = !DYN;
    constexpr int U = UB > 0 ? UB : kBatchDefault;
    const int nb = DYN ? a.nb : B;
    const int VL = DYN ? (1 << vl_log2) : (B / VPT);
    const int vls = DYN ? vl_log2 : __builtin_ctz(B / VPT);

    // the diagonal entry from the row's own x (see the gathers below): kernels with compile-time
    // flags whose lanes gather 32 bytes
    constexpr bool kDiagXin = FL != 0 && VPT * int(sizeof(X)) >= 32;
    const int C = a.C;
    const int32_t cshift = a.cshift;
    const SELL_GLOBAL int32_t *__restrict__ perm = to_global(a.perm);
    const SELL_GLOBAL int32_t *__restrict__ clp = to_global(a.cl);
    const SELL_GLOBAL int64_t *__restrict__ csp = to_global(a.cs);
    const SELL_GLOBAL int32_t *__restrict__ tiles = to_global(a.tiles);
    const int64_t nrows = a.nrows;
    // STG: the work units are the stage tiles (a.st_ntiles of a.st_chunks chunks), taken one at
    // a time: the contiguous range of units [t0, t1) of this workgroup, or with a unit stride S
    // the units Y + S k, k in [k0, k1), of column Y = tile % S one after another (on a matrix
    // whose far neighbours lie S units away, such as the next plane of a 3D grid, each unit
    // then needs much of what the previous one loaded). Otherwise the workgroup's tiles form one
    // contiguous range of slots.
    const int S = STG ? a.tile_stride : 0;
    const int64_t uch = STG ? int64_t(a.st_chunks) : 0;
    const int64_t nunits = STG ? (a.nch + uch - 1) / uch : int64_t(a.ntiles);
    int64_t r_first, r_count, r_step;  // unit i: r_first + i r_step (STG)
    if (S > 0) {
        const int64_t Q = nunits / S, nseg = a.nblocks / S, q = tile / S;
        const int64_t k0 = q * Q / nseg, k1 = (q + 1) * Q / nseg;
        r_first = (tile % S) + S * k0;
        r_count = k1 - k0;
        r_step = S;
    } else {
        const int64_t t0 = int64_t(tile) * nunits / a.nblocks, t1 = int64_t(tile + 1) * nunits / a.nblocks;
        r_first = t0;
        r_count = t1 - t0;
        r_step = 1;
    }
    // slots of unit u (STG)
    auto unit_slots = [&](int64_t u, int64_t &sb, int64_t &se) {
        const int64_t nch = a.nch;
        const int64_t c0 = u * uch, c1 = (u + 1) * uch;
        sb = (c0 < nch ? c0 : nch) * C;
        se = (c1 < nch ? c1 : nch) * C;
    };
    int64_t s_begin = 0, s_end = 0;
    const int tid = threadIdx.x;
    const int vg = tid & (VL - 1);
    const int rows_per_pass = kBlock >> vls;
    const int jb = vg * VPT;
    const bool col_ok = DYN ? (vg < nb) : true;

    const SELL_GLOBAL V *__restrict__ val = to_global(static_cast<const V *>(a.val));
    const SELL_GLOBAL int32_t *__restrict__ col = to_global(a.col);
    const SELL_GLOBAL X *__restrict__ Xp = to_global(static_cast<const X *>(a.X));
    SELL_GLOBAL X *__restrict__ Yp = to_global(static_cast<X *>(a.Y));
    SELL_GLOBAL X *__restrict__ Zp = to_global(static_cast<X *>(a.Z));
    const int64_t xrs = a.xrs, xcs = VEC ? 1 : a.xcs;
    const int64_t yrs = a.yrs, ycs = VEC ? 1 : a.ycs;
    const int64_t zrs = a.zrs, zcs = VEC ? 1 : a.zcs;

    const uint32_t fl = FL ? FL : a.flags;
    const bool want_dots = AUG && (fl & SELL_SPMV_DOTS);
    const bool shift = AUG && (fl & (SELL_SPMV_SHIFT | SELL_SPMV_VSHIFT));
    const bool need_x = shift || (AUG && (fl & (SELL_SPMV_DOT_XY | SELL_SPMV_DOT_XX)));
    const bool read_y = AUG && (fl & SELL_SPMV_AXPBY) && a.beta != 0.0;
    const bool chain = AUG && (fl & SELL_SPMV_CHAIN);
    const bool read_z = chain && a.delta != 0.0;
    const bool dot_xx = AUG && (fl & SELL_SPMV_DOT_XX);
    const bool vshift = AUG && (fl & SELL_SPMV_VSHIFT);
    const double alpha = (AUG && (fl & SELL_SPMV_SCALE)) ? a.alpha : 1.0;
    const double beta = a.beta, delta = a.delta, eta = a.eta;
    SELL_GLOBAL X *const scratch_base = to_global(static_cast<X *>(a.scratch));

    double dyy[VPT], dxy[VPT], dxx[VPT];
#pragma unroll
    for (int t = 0; t < VPT; ++t) dyy[t] = dxy[t] = dxx[t] = 0.0;

    // ---- LDS page cache of x (STG): NS slots of kStagePage rows of RB bytes. The slot of every
    // page of every unit and the pages a unit loads come from a plan made for this launch
    // shape (a.st_slot, a.st_miss). Wave 0 copies the next unit's missing pages into their
    // slots by asynchronous global-to-LDS loads, and its page -> slot table into the other half
    // of slot_tab, while the workgroup works on the current unit; the barrier that ends a unit
    // (after wave 0 has waited for its copies) makes them visible.
    constexpr int RB = (B > 0 ? B : 1) * int(sizeof(X));
    constexpr int NS_ = kStageBytes / (kStagePage * RB);
    constexpr int NS = STG ? (NS_ < kStageMaxPages ? NS_ : kStageMaxPages) : 1;
    constexpr int PGB = kStagePage * RB;  // bytes per page
    __shared__ __attribute__((aligned(16))) unsigned char cache[STG ? NS * PGB : 16];
    __shared__ int32_t slot_tab[STG ? 2 : 1][STG ? kStageMaxPages : 1];  // slot of a unit's i-th page
    const int lane = tid & 63;
    // Wave 0: start loading unit ub's missing pages (npb pages listed) and its slot table into
    // slot_tab[half]. The caller waits for the copies (s_waitcnt) and then synchronises the
    // workgroup before either is read.
    auto load_unit = [&](int64_t ub, int npb, int half_) {
        const SELL_GLOBAL int8_t *sp = to_global(a.st_slot) + ub * kStageMaxPages;
        const SELL_GLOBAL int32_t *pl = to_global(a.st_pages) + ub * kStageMaxPages;
        if (lane < npb) slot_tab[half_][lane] = sp[lane];
        const SELL_GLOBAL unsigned char *xb = reinterpret_cast<const SELL_GLOBAL unsigned char *>(Xp);
        const int64_t xbytes = a.ncols_x * RB;
        uint64_t todo = to_global(a.st_miss)[ub];
        while (todo) {
            const int k = __builtin_ctzll(todo);
            todo &= todo - 1;
            const int64_t goff = int64_t(pl[k]) * PGB;
            const int sl = sp[k];
#pragma unroll
            for (int q = 0; q < (PGB + 1023) / 1024; ++q) {
                const int o = q * 1024 + lane * 16;
                if (o < PGB && goff + o + 16 <= xbytes)
                    __builtin_amdgcn_global_load_lds(xb + goff + o,
                                                     (__attribute__((address_space(3))) void *)(cache + sl * PGB + q * 1024),
                                                     16, 0, 0);
            }
        }
    };

    double gam[VPT];
#pragma unroll
    for (int t = 0; t < VPT; ++t) gam[t] = (vshift && a.has_gamma_v && col_ok) ? a.gamma_v[jb + t] : a.gamma_s;

    // Chunk metadata of a slot, loaded one pass ahead. The loads are unconditional (the slot
    // is clamped into the tile, and without a permutation the row load re-reads the chunk
    // length) and nothing is computed from them until the next pass, so their latency
    // overlaps the current pass.
    auto load_meta = [&](int64_t ss, int64_t se_, int &clv, int64_t &csv, int &pv) {
        const int64_t sc = ss < se_ ? ss : se_ - 1;
        const int64_t c = cshift >= 0 ? (sc >> cshift) : int64_t(uint32_t(sc) / uint32_t(C));
        const SELL_GLOBAL int32_t *pp = perm ? perm + sc : clp + c;
        clv = clp[c];
        csv = csp[c];
        pv = *pp;
    };

    // One pass: the lanes' slot s (row `row`, -1 for none) with len entries at base; with x
    // staged (staged), gathers read the LDS cache through slot_tab[half], and the own rows'
    // x from their pages (own_pos: list position of the page of the unit's first row,
    // own_p0 that page).
    auto pass_body = [&](const int64_t s, const int len, const int64_t base, const int64_t row, const bool staged,
                         const int own_pos, const int64_t own_p0, const int half) {
        const bool live = row >= 0 && col_ok;
        // Lanes without an output row (slots past the last row, or unused columns of the
        // generic kernel) read row 0 / column 0 and store into the scratch area, so no load
        // or store of a pass sits under a divergent branch.
        const int64_t rowc = live ? row : 0;
        const int jl = col_ok ? jb : 0;

        // epilogue operands, issued before the gathers so their latency overlaps
        X xin[VPT], yin[VPT], zin[VPT];
#pragma unroll
        for (int t = 0; t < VPT; ++t) xin[t] = yin[t] = zin[t] = X(0);
        if (AUG) {
            if (STG && staged && own_pos >= 0 && need_x) {
                const int pos = own_pos + int((rowc >> kStagePageShift) - own_p0);
                const int sl = live ? slot_tab[half][pos] : slot_tab[half][own_pos];
                const X *src = reinterpret_cast<const X *>(cache + ((sl << kStagePageShift) | int(rowc & (kStagePage - 1))) * RB) + jb;
#pragma unroll
                for (int t = 0; t < VPT; ++t) xin[t] = src[t];
            } else if (need_x) load_row<X, VPT, VEC>(Xp + rowc * xrs + int64_t(jl) * xcs, xcs, xin);
            if (read_y) load_row<X, VPT, VEC>(Yp + rowc * yrs + int64_t(jl) * ycs, ycs, yin);
            if (read_z) load_row<X, VPT, VEC>(Zp + rowc * zrs + int64_t(jl) * zcs, zcs, zin);
        }

        Acc acc[VPT];
#pragma unroll
        for (int t = 0; t < VPT; ++t) acc[t] = Acc(0);
        if (col_ok) {
            for (int k0 = 0; k0 < len; k0 += U) {
                int ci[U];
                V vv[U];
                X xg[U][VPT];
                if (STG && staged) {
                    // tile-local indices (page position, row in page), gathered from the cache
                    const SELL_GLOBAL uint16_t *__restrict__ lcol = to_global(a.lcol);
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int k = min(k0 + u, len - 1);
                        const int64_t at = base + int64_t(k) * C;
                        const int lc = __builtin_nontemporal_load(lcol + at);
                        const V v = __builtin_nontemporal_load(val + at);
                        ci[u] = (k0 + u < len && lc != 0xFFFF) ? lc : -1;
                        vv[u] = v;
                    }
                    int sl[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) sl[u] = slot_tab[half][(ci[u] >= 0 ? ci[u] : 0) >> kStagePageShift];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int lr = (sl[u] << kStagePageShift) | ((ci[u] >= 0 ? ci[u] : 0) & (kStagePage - 1));
                        const X *src = reinterpret_cast<const X *>(cache + lr * RB) + jb;
#pragma unroll
                        for (int t = 0; t < VPT; ++t) xg[u][t] = src[t];
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        // clamp to the row's last entry so every load is in bounds and unconditional
                        const int k = min(k0 + u, len - 1);
                        const int64_t at = base + int64_t(k) * C;
                        const int cc = __builtin_nontemporal_load(col + at);
                        const V v = __builtin_nontemporal_load(val + at);
                        ci[u] = (k0 + u < len) ? cc : -1;
                        vv[u] = v;
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int cu = ci[u] >= 0 ? ci[u] : 0;  // padding / tail: harmless in-bounds gather
                        if (AUG && kDiagXin && need_x && int64_t(cu) == rowc) {
                            // the diagonal entry: the row's own x is in xin already (loaded for the
                            // shift and the dots), so this lane's gather is masked off and the
                            // CU's vector memory path carries 1/len less (128.4 against 132.8 us
                            // for the KPM product on the 128^3 Anderson matrix at b = 8). With
                            // 16-byte gathers the branch costs what it saves, and in the kernels
                            // with run-time flags it costs more (the 100^3 Laplacian with <x,y>
                            // at b = 8: 64 -> 71 us; the 64-Laplacian batch 1336 -> 1405 us), so
                            // only the compile-time-flag kernels that gather 32 bytes take it)
#pragma unroll
                            for (int t = 0; t < VPT; ++t) xg[u][t] = xin[t];
                        } else {
                            load_row<X, VPT, VEC>(Xp + int64_t(cu) * xrs + int64_t(jb) * xcs, xcs, xg[u]);
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const Acc v = to_acc(vv[u], Acc(0));
#pragma unroll
                    for (int t = 0; t < VPT; ++t) {
                        const Acc f = fmadd(v, Acc(xg[u][t]), acc[t]);
                        acc[t] = ci[u] >= 0 ? f : acc[t];
                    }
                }
            }
        }

        SELL_GLOBAL X *scratch = scratch_base + size_t(tid) * VPT;
        SELL_GLOBAL X *ydst = live ? Yp + row * yrs + int64_t(jb) * ycs : scratch;
        const int64_t ysd = live ? ycs : 1;
        X out[VPT];
        if (!AUG) {
#pragma unroll
            for (int t = 0; t < VPT; ++t) out[t] = X(acc[t]);
            store_row<X, VPT, VEC>(ydst, ysd, out);
        } else {
            X zout[VPT];
#pragma unroll
            for (int t = 0; t < VPT; ++t) {
                const double xv = double(xin[t]);
                double tv = double(acc[t]);
                if (shift) tv = tv - gam[t] * xv;
                double y = alpha * tv;
                if (read_y) y = y + beta * double(yin[t]);
                out[t] = X(y);
                const double yd = double(out[t]);
                if (want_dots && live) {
                    dyy[t] += yd * yd;
                    dxy[t] += xv * yd;
                    if (dot_xx) dxx[t] += xv * xv;
                }
                double z = eta * yd;
                if (read_z) z = delta * double(zin[t]) + z;
                zout[t] = X(z);
            }
            store_row<X, VPT, VEC>(ydst, ysd, out);
            if (chain) {
                SELL_GLOBAL X *zdst = live ? Zp + row * zrs + int64_t(jb) * zcs : scratch;
                store_row<X, VPT, VEC>(zdst, live ? zcs : 1, zout);
            }
        }
    };

    if constexpr (!STG) {
        const int64_t t0 = int64_t(tile) * a.ntiles / a.nblocks, t1 = int64_t(tile + 1) * a.ntiles / a.nblocks;
        s_begin = int64_t(tiles[t0]) * C;
        s_end = int64_t(tiles[t1]) * C;
        int64_t s = s_begin + (tid >> vls);
        int cl_n = 0, pv_n = 0;
        int64_t cs_n = 0;
        if (s_begin < s_end) load_meta(s, s_end, cl_n, cs_n, pv_n);
        // Settle the first pass's metadata here, so that at the loop head only the previous
        // pass's stores are outstanding and the metadata loads of the following pass are not
        // held up behind them.
        __builtin_amdgcn_s_waitcnt(0);
        for (; s < s_end; s += rows_per_pass) {
            const int64_t c = cshift >= 0 ? (s >> cshift) : int64_t(uint32_t(s) / uint32_t(C));
            const int len = cl_n;
            const int64_t base = cs_n + (s - c * C);
            const int64_t row = s < nrows ? (perm ? int64_t(pv_n) : s) : -1;
            load_meta(s + rows_per_pass, s_end, cl_n, cs_n, pv_n);  // one pass ahead
            pass_body(s, len, base, row, false, -1, 0, 0);
        }
    } else {
        // The workgroup's passes over all of its units, one after another: the metadata of the next
        // pass (in this unit or at the start of the next) is loaded one pass ahead.
        // STG: a unit's pages are resident and listed in slot_tab[half] when its first pass starts;
        // the first unit is staged here, each next one during the unit before it when both fit.
        int half = 0;
        auto unit_np = [&](int64_t u) {
            const int n = a.st_np[u];
            return (n > 0 && n <= NS) ? n : 0;
        };
        int64_t rr = 0;
        if (r_count > 0) unit_slots(r_first, s_begin, s_end);
        if constexpr (STG) {
            if (r_count > 0) {
                const int n0 = unit_np(r_first);
                if (n0 > 0) {
                    if (tid < 64) {
                        load_unit(r_first, n0, 0);
                        __builtin_amdgcn_s_waitcnt(0);
                    }
                    __syncthreads();
                }
            }
        }
        int64_t pb = s_begin;  // first slot of the current pass
        int cl_n = 0, pv_n = 0;
        int64_t cs_n = 0;
        if (r_count > 0 && s_begin < s_end) load_meta(pb + (tid >> vls), s_end, cl_n, cs_n, pv_n);
        // Settle the first pass's metadata here, so that at the loop head only the previous
        // pass's stores are outstanding and the metadata loads of the following pass are not
        // held up behind them.
        __builtin_amdgcn_s_waitcnt(0);
        bool staged = false, ahead = false;
        int own_pos = -1, np_next = 0;
        int64_t tb = 0, own_p0 = 0;
        while (rr < r_count) {
            const int64_t ta = r_first + rr * r_step;
            if (pb == s_begin) {
                // first pass of unit ta
                if constexpr (STG) {
                    const int npa = unit_np(ta);
                    staged = npa > 0;
                    own_pos = staged ? a.st_own[ta] : -1;
                    ahead = false;
                    np_next = 0;
                    if (rr + 1 < r_count) {
                        tb = ta + r_step;
                        np_next = unit_np(tb);
                        // the next unit's pages load during this one when both fit the cache together
                        ahead = np_next > 0 && npa + np_next <= NS;
                        if (ahead && tid < 64) load_unit(tb, np_next, half ^ 1);
                    }
                }
                // list position of the page of the unit's first row (own rows read x from the cache)
                own_p0 = s_begin >> kStagePageShift;
            }
            // the following pass: in this unit, or the first pass of the next one
            int64_t nrr = rr, nsb = s_begin, nse = s_end, npb = pb + rows_per_pass;
            if (npb >= s_end) {
                nrr = rr + 1;
                if (nrr < r_count) {
                    unit_slots(r_first + nrr * r_step, nsb, nse);
                    npb = nsb;
                }
            }
            const int64_t s = pb + (tid >> vls);
            const int64_t c = cshift >= 0 ? (s >> cshift) : int64_t(uint32_t(s) / uint32_t(C));
            const int len = s < s_end ? cl_n : 0;
            const int64_t base = cs_n + (s - c * C);
            const int64_t row = s < s_end && s < nrows ? (perm ? int64_t(pv_n) : s) : -1;
            if (nrr < r_count && nsb < nse) load_meta(npb + (tid >> vls), nse, cl_n, cs_n, pv_n);  // one pass ahead
            pass_body(s, len, base, row, staged, own_pos, own_p0, half);
            if (nrr != rr) {
                // last pass of unit ta
                if constexpr (STG) {
                    if (ahead) {
                        // wave 0's copies of the next unit's pages must land before anyone reads them
                        if (tid < 64) __builtin_amdgcn_s_waitcnt(0);
                        __syncthreads();
                        half ^= 1;
                    } else if (np_next > 0) {
                        // the next unit's pages did not fit beside this unit's: load them now
                        __syncthreads();
                        if (tid < 64) {
                            load_unit(tb, np_next, half ^ 1);
                            __builtin_amdgcn_s_waitcnt(0);
                        }
                        __syncthreads();
                        half ^= 1;
                    }
                }
                s_begin = nsb;
                s_end = nse;
            }
            rr = nrr;
            pb = npb;
        }  // passes
    }

    if (!want_dots) return;

    // ---- dot partials of this tile (deterministic: butterfly in the wave, waves in order)
    __shared__ double red[kBlock / 64][3 * kMaxSliceCols];
    const int w = tid >> 6;
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
    // one partial per tile and quantity, plain stores: the sums over tiles are taken by a
    // separate kernel (kernel boundaries order the memory without device-wide fences)
    const int nq = 3 * nb;
    for (int q = tid; q < nq; q += kBlock) {
        double sum = 0.0;
#pragma unroll
        for (int ww = 0; ww < kBlock / 64; ++ww) sum += red[ww][q];
        to_global(a.partials)[size_t(q) * a.nblocks + tile] = sum;
    }
}

template <int VK, int B, int VPT, bool AUG, int UB = 0, bool STG = false, uint32_t FL = 0>
__global__ void __launch_bounds__(kBlock) prod_kernel(ProdArgs a, int vl_log2) {
    const int tile = a.xcd_map ? xcd_tile(blockIdx.x, gridDim.x) : int(blockIdx.x);  // index in the partials
    int vls = vl_log2;
    if (B == 0 && vls < 0) {
        vls = 0;
        while ((1 << vls) < a.nb) ++vls;
    }
    prod_body<VK, B, VPT, AUG, UB, STG, FL>(a, tile, vls);
}

// The flags of a step of the Chebyshev / KPM recurrence (y = alpha (A x - c x) - y with
// <y, y> and <x, y>): the FP64 product the KPM driver runs M times gets its own compile-time
// copy (130 VGPRs against 160 for the general epilogue; 133.9 against 135.8 us per product on
// the 128^3 Anderson matrix at b = 8). Forcing it to 128 VGPRs for two workgroups per compute
// unit (amdgpu_waves_per_eu(4)) spills a register and is slower (142.5 against 138.0 us per
// call with its dot finish).
constexpr uint32_t kKpmFlags = SELL_SPMV_SHIFT | SELL_SPMV_SCALE | SELL_SPMV_AXPBY | SELL_SPMV_DOT_YY | SELL_SPMV_DOT_XY;

// The flags of a CG iteration's product (q = A p with <q, q> and <p, q>): the FP32-vector kernels
// (FP32 or BF16 values, the mixed-precision solvers' inner iterations) get their own compile-time
// copy, single-matrix and batched (100^3 Laplacian, BF16 values, b = 8, with <p, q> alone:
// 36.0 -> 33.7 us). The FP64 kernel gained nothing from it (64.1 against 65.0 us) and keeps the
// run-time flags.
constexpr uint32_t kCgFlags = SELL_SPMV_DOT_YY | SELL_SPMV_DOT_XY;

// One launch over a batch of matrices: workgroups [blk_start[m], blk_start[m+1]) of the
// (XCD-remapped) grid work on matrix m, whose launch arguments are table[m]. A matrix m with
// active != null and active[m] == 0 is skipped (its dot partials are zeroed). With the
// run-time-width kernel (B == 0) and vl_log2 < 0 every matrix gets the lanes per row of its
// own width (table[m].nb), so matrices of different block widths share the launch.
template <int VK, int B, int VPT, bool AUG, int UB = 0, uint32_t FL = 0>
__global__ void __launch_bounds__(kBlock) prod_batch_kernel(const ProdArgs *__restrict__ table,
                                                            const int32_t *__restrict__ blk_start, int K,
                                                            const int32_t *__restrict__ active, int vl_log2) {
    const int g = xcd_tile(blockIdx.x, gridDim.x);
    int lo = 0, hi = K;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (blk_start[mid] <= g)
            lo = mid;
        else
            hi = mid;
    }
    const ProdArgs &a = table[lo];
    const int tile = g - blk_start[lo];
    if (active && !active[lo]) {
        if (AUG && (a.flags & SELL_SPMV_DOTS))
            for (int q = threadIdx.x; q < 3 * a.nb; q += kBlock) to_global(a.partials)[size_t(q) * a.nblocks + tile] = 0.0;
        return;
    }
    int vls = vl_log2;
    if (B == 0 && vls < 0) {
        vls = 0;
        while ((1 << vls) < a.nb) ++vls;
    }
    prod_body<VK, B, VPT, AUG, UB, false, FL>(a, tile, vls);
}

// A batch whose matrices have block widths of their own, in one launch: every workgroup runs
// the body compiled for its matrix's width (1, 2, 4, 8, 16 or 32, with the default columns
// per lane), or the run-time-width body for any other width or for operands whose rows do
// not allow vector accesses (runtime_width). The branch depends only on the workgroup's
// matrix, so it is uniform over the workgroup.
template <int VK, bool AUG>
__global__ void __launch_bounds__(kBlock) prod_batch_mixed_kernel(const ProdArgs *__restrict__ table,
                                                                  const int32_t *__restrict__ blk_start, int K,
                                                                  const int32_t *__restrict__ active, int) {
    const int g = xcd_tile(blockIdx.x, gridDim.x);
    int lo = 0, hi = K;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (blk_start[mid] <= g)
            lo = mid;
        else
            hi = mid;
    }
    const ProdArgs &a = table[lo];
    const int tile = g - blk_start[lo];
    if (active && !active[lo]) {
        if (AUG && (a.flags & SELL_SPMV_DOTS))
            for (int q = threadIdx.x; q < 3 * a.nb; q += kBlock) to_global(a.partials)[size_t(q) * a.nblocks + tile] = 0.0;
        return;
    }
    switch (a.runtime_width ? 0 : a.nb) {
        case 1: prod_body<VK, 1, 1, AUG>(a, tile, 0); break;
        case 2: prod_body<VK, 2, 2, AUG>(a, tile, 0); break;
        case 4: prod_body<VK, 4, 4, AUG>(a, tile, 0); break;
        case 8: prod_body<VK, 8, 4, AUG>(a, tile, 0); break;
        case 16: prod_body<VK, 16, 4, AUG>(a, tile, 0); break;
        case 32: prod_body<VK, 32, 4, AUG>(a, tile, 0); break;
        default: {
            int vls = 0;
            while ((1 << vls) < a.nb) ++vls;
            prod_body<VK, 0, 1, AUG>(a, tile, vls);
        }
    }
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
    const int tile = a.xcd_map ? xcd_tile(blockIdx.x, gridDim.x) : int(blockIdx.x);
    const int C = a.C;
    const int64_t t0 = int64_t(tile) * a.ntiles / a.nblocks, t1 = int64_t(tile + 1) * a.ntiles / a.nblocks;
    const int64_t s_begin = int64_t(a.tiles[t0]) * C;
    const int64_t s_end = int64_t(a.tiles[t1]) * C;
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

template <int VK, int B, int VPT, bool AUG, int UB = 0>
inline int go_prod_u(ProdArgs &a, hipStream_t s) {
    int vl_log2 = 0;
    if (B == 0) {
        while ((1 << vl_log2) < a.nb) ++vl_log2;
    }
    using X = typename KTypes<VK>::X;
    // x through the LDS page cache: fixed widths over contiguous, 16-byte aligned rows
    if (a.stage && !(B > 0 && B * sizeof(X) >= 16 && a.xrs == B && a.xcs == 1 && a.lcol && a.st_slot &&
                     (reinterpret_cast<uintptr_t>(a.X) & 15u) == 0))
        a.stage = 0;
    auto k = a.stage ? prod_kernel<VK, B, VPT, AUG, UB, (B > 0)> : prod_kernel<VK, B, VPT, AUG, UB>;
    if constexpr (AUG && VK == VK_F64F64 && B > 0) {
        if (!a.stage && a.flags == kKpmFlags)
            k = prod_kernel<VK, B, VPT, AUG, UB, false, kKpmFlags>;
    }
    if constexpr (AUG && VK != VK_F64F64 && B > 0) {
        if (!a.stage && a.flags == kCgFlags)
            k = prod_kernel<VK, B, VPT, AUG, UB, false, kCgFlags>;
    }
    if (a.stage) {
        a.nblocks = a.st_nblocks;  // the launch the plan was made for (stride checked there)
        hipLaunchKernelGGL(k, dim3(a.nblocks), dim3(kBlock), 0, s, a, vl_log2);
        return hipGetLastError() == hipSuccess ? SELL_OK : SELL_ERR_HIP;
    }
    // Lanes that gather 32 bytes per entry (FP64 rows, 4 columns per lane) run one workgroup per
    // compute unit unless the caller chose (sell_set_launch): more waves of such gathers per CU
    // slow the CU's vector memory path down (plain FP64 products at b = 8 / 16 / 32: 113 / 220 /
    // 462 us with two workgroups per CU on the 128^3 Anderson matrix, 103 / 202 / 423 with one;
    // FP32 vectors, 16 bytes per lane, stay faster with two).
    int32_t bpc = a.bpc_hint;
    if (bpc == 0 && VPT * int(sizeof(typename KTypes<VK>::X)) >= 32) bpc = 1;
    a.nblocks = resident_grid(reinterpret_cast<const void *>(k), kBlock, a.ntiles, bpc);
    // several waves: workgroups that finish early take the next ones (uneven tiles)
    if (a.waves_hint > 1) a.nblocks = int32_t(std::min<int64_t>(int64_t(a.nblocks) * a.waves_hint, a.ntiles));
    // a tile stride needs whole columns of tiles and of workgroups
    a.tile_stride = 0;  // a unit stride applies to staged launches only
    hipLaunchKernelGGL(k, dim3(a.nblocks), dim3(kBlock), 0, s, a, vl_log2);
    return hipGetLastError() == hipSuccess ? SELL_OK : SELL_ERR_HIP;
}

// The fixed-width kernels of 8-entry index batches come with batches of 5 and 7 as well: a
// batch is issued whole, so a chunk of L entries costs ceil(L / U) rounds of U loads, and
// 7- or 5-entry batches waste no loads on rows of 7 or 5 entries (3D and 2D stencils). The
// matrix's batch_hint (chosen from its chunk lengths, or set by the caller) picks one.
template <int VK, int B, int VPT, bool AUG>
inline int go_prod(ProdArgs &a, hipStream_t s) {
    using X = typename KTypes<VK>::X;
    if constexpr (B > 0) {
        const int hint = VPT * sizeof(X) >= 32 ? a.batch_hint_wide : a.batch_hint;
        if (hint == 7) return go_prod_u<VK, B, VPT, AUG, 7>(a, s);
        if (hint == 5) return go_prod_u<VK, B, VPT, AUG, 5>(a, s);
    }
    return go_prod_u<VK, B, VPT, AUG>(a, s);
}

template <int VK, int B, int VPT>
inline int go_transpose(ProdArgs &a, hipStream_t s) {
    int vl_log2 = 0;
    if (B == 0) {
        while ((1 << vl_log2) < a.nb) ++vl_log2;
    }
    auto k = transpose_kernel<VK, B, VPT>;
    a.nblocks = resident_grid(reinterpret_cast<const void *>(k), kBlock, a.ntiles);
    hipLaunchKernelGGL(k, dim3(a.nblocks), dim3(kBlock), 0, s, a, vl_log2);
    return hipGetLastError() == hipSuccess ? SELL_OK : SELL_ERR_HIP;
}


template <int VK, bool AUG>
int dispatch_prod(ProdArgs &a, hipStream_t s, bool fixed_ok) {
    const int b = a.nb;
    const int vpt = choose_vpt(VK, b, a.vpt_hint);
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

template <int VK, int B, int VPT, bool AUG, int UB = 0>
inline const void *bk_u(bool cg) {
    if constexpr (AUG && VK != VK_F64F64 && B > 0) {
        if (cg) return reinterpret_cast<const void *>(prod_batch_kernel<VK, B, VPT, AUG, UB, kCgFlags>);
    }
    return reinterpret_cast<const void *>(prod_batch_kernel<VK, B, VPT, AUG, UB>);
}

// The batched kernel of index batch length ub (ubw for the kernels gathering 32 bytes per
// lane; 5 or 7 where the width's default is 8, as for the single-matrix kernels; else the
// default)
template <int VK, int B, int VPT, bool AUG>
inline const void *bk(int ub0, int ubw, bool cg) {
    using X = typename KTypes<VK>::X;
    if constexpr (B > 0) {
        const int ub = VPT * sizeof(X) >= 32 ? ubw : ub0;
        if (ub == 7) return bk_u<VK, B, VPT, AUG, 7>(cg);
        if (ub == 5) return bk_u<VK, B, VPT, AUG, 5>(cg);
    }
    return bk_u<VK, B, VPT, AUG>(cg);
}

// The batched kernel for (width, columns per lane, index batch length); fixed_ok as in
// dispatch_prod.
template <int VK, bool AUG>
const void *batch_kernel_for(int b, int vpt, bool fixed_ok, int ub, int ubw, uint32_t flags) {
    const bool cg = flags == kCgFlags;
    if (fixed_ok) {
        switch (b) {
            case 1: return bk<VK, 1, 1, AUG>(ub, ubw, cg);
            case 2: return vpt >= 2 ? bk<VK, 2, 2, AUG>(ub, ubw, cg) : bk<VK, 2, 1, AUG>(ub, ubw, cg);
            case 4: return vpt >= 4 ? bk<VK, 4, 4, AUG>(ub, ubw, cg) : vpt == 2 ? bk<VK, 4, 2, AUG>(ub, ubw, cg) : bk<VK, 4, 1, AUG>(ub, ubw, cg);
            case 8: return vpt >= 4 ? bk<VK, 8, 4, AUG>(ub, ubw, cg) : vpt == 2 ? bk<VK, 8, 2, AUG>(ub, ubw, cg) : bk<VK, 8, 1, AUG>(ub, ubw, cg);
            case 16:
                return vpt >= 4 ? bk<VK, 16, 4, AUG>(ub, ubw, cg) : vpt == 2 ? bk<VK, 16, 2, AUG>(ub, ubw, cg) : bk<VK, 16, 1, AUG>(ub, ubw, cg);
            case 32:
                return vpt >= 4 ? bk<VK, 32, 4, AUG>(ub, ubw, cg) : vpt == 2 ? bk<VK, 32, 2, AUG>(ub, ubw, cg) : bk<VK, 32, 1, AUG>(ub, ubw, cg);
            default: break;
        }
    }
    return bk<VK, 0, 1, AUG>(ub, ubw, cg);
}

template <int VK, bool AUG>
const void *batch_mixed_kernel_for() {
    return reinterpret_cast<const void *>(prod_batch_mixed_kernel<VK, AUG>);
}

template <int VK>
int dispatch_transpose(ProdArgs &a, hipStream_t s) {
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
