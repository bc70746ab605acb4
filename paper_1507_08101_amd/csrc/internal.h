// internal.h -- shared definitions of libsellcs (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <memory>
#include <vector>

#include "sellcs.h"

namespace sellcs {

constexpr int kMaxSliceCols = 64;   // widest column slice one product launch handles
constexpr int kMaxTiles = 4096;     // upper bound on work partitions per launch
constexpr int kBlock = 512;         // threads per block of the product kernels
// Gathering x through LDS: x rows in pages of kStagePage rows; a tile is staged when it
// references at most kStageMaxPages pages; the page cache of a workgroup holds kStageBytes.
constexpr int kStagePageShift = 6;
constexpr int kStagePage = 1 << kStagePageShift;
constexpr int kStageMaxPages = 64;
constexpr int kStageBytes = 144 * 1024;

inline int dtype_bytes(int dt) { return dt == SELL_F64 ? 8 : dt == SELL_F32 ? 4 : 2; }

// Allocator that leaves new elements uninitialised (the builder writes every element itself,
// in parallel, so a serial zero fill of hundreds of MB is saved).
template <class T>
struct NoInitAlloc : std::allocator<T> {
    template <class U>
    struct rebind {
        using other = NoInitAlloc<U>;
    };
    NoInitAlloc() = default;
    template <class U>
    NoInitAlloc(const NoInitAlloc<U> &) noexcept {}
    template <class U>
    void construct(U *p) noexcept {
        ::new (static_cast<void *>(p)) U;
    }
    template <class U, class... A>
    void construct(U *p, A &&...a) {
        ::new (static_cast<void *>(p)) U(std::forward<A>(a)...);
    }
};
template <class T>
using raw_vector = std::vector<T, NoInitAlloc<T>>;

// Host-side SELL-C-sigma arrays (the build result before upload).
struct HostSell {
    int64_t nrows = 0, ncols = 0, nnz = 0, stored = 0, nch = 0, sigma = 1;
    int32_t C = 1;
    int vdt = SELL_F64;
    bool has_perm = false;
    std::vector<int32_t> perm;    // slot -> row (-1 past the end); empty when identity
    std::vector<int32_t> cl;      // chunk lengths
    std::vector<int64_t> cs;      // chunk starts (nch + 1)
    raw_vector<int32_t> col;      // stored column indices (-1 = padding)
    raw_vector<uint8_t> val;      // stored values in storage type
    std::vector<int32_t> tiles;   // ntiles + 1 chunk boundaries
    std::vector<int64_t> rowptr;  // CSR row pointers of the input (for export and updates)
    int32_t batch = 8;            // index batch length suited to the chunk lengths (5, 7 or 8)
    int32_t batch_wide = 7;       // the same for the kernels gathering 32 bytes per lane (5 or 7)
    int32_t waves = 1;            // default product grid in waves of resident workgroups (1 or 16)
};

// Work partitions: contiguous chunk ranges of roughly equal cost.
int32_t default_tile_count(int64_t nch);
void make_tiles(const std::vector<int32_t> &cl, int32_t C, int32_t ntiles,
                std::vector<int32_t> &tiles);

// Index batch length (5, 7 or 8) for the product kernels, from the chunk lengths: a chunk of
// L entries costs ceil(L / U) batch rounds of U loads each plus a fixed cost per round. wide:
// for the kernels whose lane gathers 32 bytes per entry, where 8-entry batches leave room for
// two waves per SIMD instead of three: 5 or 7 only.
int32_t choose_batch_len(const std::vector<int32_t> &cl, bool wide = false);
// Default product grid in waves of resident workgroups from the spread of the chunk lengths.
int32_t choose_waves(const std::vector<int32_t> &cl);

// Validates CSR input and builds the host SELL arrays. Returns SELL_OK or an error.
int build_host_sell(HostSell &h, int64_t nrows, int64_t ncols, const int64_t *rowptr,
                    const int32_t *col, const double *val, int32_t C, int64_t sigma, int vdt);

}  // namespace sellcs
struct sell_mat;
namespace sellcs {
// Builds the SELL arrays on the device from a CSR matrix in device memory (devbuild.hip);
// fills the device arrays and the host metadata of M. On error M may hold device arrays.
int build_device_sell(sell_mat *M, int64_t nrows, int64_t ncols, const int64_t *rowptr, const int32_t *col,
                      const double *val, int32_t C, int64_t sigma, int vdt, hipStream_t s);

// Value conversion (round to nearest, ties to even, from the double).
uint16_t f64_to_bf16_bits(double v);
float bf16_bits_to_f32(uint16_t b);
void convert_values(const double *src, int64_t n, int vdt, void *dst);

}  // namespace sellcs

struct sell_mat {
    sellcs::HostSell h;           // metadata always; col/val only for host-only builds
    bool on_device = false;
    int device = -1;
    int32_t ntiles = 0;
    int32_t *d_col = nullptr;
    void *d_val = nullptr;
    int32_t *d_cl = nullptr;
    int64_t *d_cs = nullptr;
    int32_t *d_perm = nullptr;    // null when rows keep their order
    int32_t *d_tiles = nullptr;
    int32_t *d_rowslot = nullptr; // row -> slot, built on first device value update
    int64_t *d_rowptr = nullptr;  // CSR row pointers, built on first device value update
    sell_mat *transpose = nullptr;  // SELL copy of A^T for the deterministic transpose
    int64_t *d_tpos = nullptr;      // position in the SELL arrays of A^T of each CSR entry of A
    // LDS staging of x (built on first use, stage.hip): per tile the page count (0: not
    // staged), the sorted page list, the list position of the tile's own first row page (-1:
    // not all own rows listed); per stored entry the tile-local column index
    int32_t *d_stage_np = nullptr;
    int32_t *d_stage_pages = nullptr;
    int32_t *d_stage_own = nullptr;
    uint16_t *d_lcol = nullptr;
    int8_t *d_plan_slot = nullptr;  // staged launch plan: slot of each page of each stage tile,
    uint64_t *d_plan_miss = nullptr;  // and the pages each tile loads, for (plan_nblk
    int32_t plan_nblk = -1, plan_stride = -1, plan_ns = -1;  // workgroups, stride, slots)
    int32_t stage_chunks = 0;       // chunks per stage tile of the arrays above
    int32_t stage_ntiles = 0;       // number of stage tiles
    int32_t stage_hint = 0;         // 1: products gather x through LDS where the tile allows
    int32_t tile_stride_hint = 0;   // > 0: workgroups take every tile_stride-th tile
    int64_t matrix_bytes = 0;
    int32_t vpt_hint = 0;           // launch parameters chosen for this matrix (0: defaults)
    int32_t bpc_hint = 0;
    int32_t slice_hint = 0;         // process wider blocks in slices of this width (0: whole)
    int32_t waves_hint = 0;         // product grid in waves of the resident workgroups (0, 1: one)
    int32_t batch_hint = 0;         // index batch length set by the caller (5, 7, 8; 0: h.batch
                                    // and h.batch_wide)
};

struct sell_bv {
    int64_t nrows = 0;
    int32_t ncols = 0;
    int dt = SELL_F64;
    int lay = SELL_ROW_MAJOR;
    void *ptr = nullptr;
    int64_t ld = 0;
    bool owned = false;
    int device = -1;
};

namespace sellcs {

// ---------------------------------------------------------------- kernel launchers
// Parameters of one product launch over a slice of columns [j0, j0 + nb).
struct ProdArgs {
    const int32_t *col;
    const void *val;
    const int32_t *cl;
    const int64_t *cs;
    const int32_t *perm;   // may be null (identity)
    const int32_t *tiles;
    int32_t ntiles, C;     // fine work partitions of the matrix; chunk height
    int32_t nblocks;       // workgroups of the launch (set by the launcher); workgroup g
                           // owns fine tiles [g * ntiles / nblocks, (g + 1) * ntiles / nblocks)
    int32_t cshift;        // log2(C) when C is a power of two, else -1
    int32_t xcd_map;       // 1: give each XCD one contiguous range of tiles
    int32_t vpt_hint;      // columns per lane requested for the matrix (0: default)
    int32_t bpc_hint;      // workgroups per compute unit requested (0: occupancy limit)
    int32_t waves_hint;    // product grid in waves of resident workgroups (0, 1: one wave)
    int32_t batch_hint;    // index batch length of the kernels (5, 7; else 8)
    int32_t batch_hint_wide; // the same for the kernels gathering 32 bytes per lane
    int32_t tile_stride;   // > 0 (staged launches): workgroup g takes every tile_stride-th
                           // stage tile of its column
    int32_t stage;         // 1: gather x through the LDS page cache (the stage arrays below)
    int32_t st_ntiles;     // stage tiles: st_chunks consecutive chunks each (the last may be short)
    int32_t st_chunks;
    int64_t nch;           // chunks of the matrix
    const int32_t *st_np, *st_pages, *st_own;
    const uint16_t *lcol;
    const int8_t *st_slot;     // the launch plan (ensure_stage_plan) for st_nblocks workgroups
    const uint64_t *st_miss;
    int32_t st_nblocks;
    int32_t runtime_width; // batched launch of mixed widths: 1 = this matrix's rows do not
                           // allow vector accesses, use the run-time-width body
    int64_t nrows;
    int64_t ncols_x;       // rows of X (columns of the matrix)
    int32_t nb;            // columns in this slice
    const void *X; int64_t xrs, xcs;   // element (i, j) at X[i * xrs + j * xcs]
    void *Y; int64_t yrs, ycs;
    void *Z; int64_t zrs, zcs;
    uint32_t flags;
    double alpha, beta, delta, eta;
    int32_t has_gamma_v;   // per-column shifts below (else the scalar gamma_s)
    double gamma_s;        // scalar shift
    double gamma_v[kMaxSliceCols];
    void *scratch;         // kBlock * 16 bytes of write-only scratch for lanes without a row
    double *partials;      // dots: 3 * nb * nblocks doubles, partials[q * nblocks + g],
                           // q = group * nb + j for group = yy, xy, xx
};

enum VecKind { VK_F64F64 = 0, VK_F32F32 = 1, VK_BF16F32 = 2 };

int launch_product(ProdArgs &a, int vk, bool aug, hipStream_t s);
int launch_transpose_atomic(ProdArgs &a, int vk, hipStream_t s);
int launch_fill(void *p, int dt, int64_t nrows, int32_t ncols, int64_t rs, int64_t cs,
                double value, hipStream_t s);
int launch_copy(const sell_bv *dst, const sell_bv *src, hipStream_t s);
int launch_update_values(const sell_mat *A, const double *val_dev, hipStream_t s);
int launch_probe(int kind, void *dst, const void *src, int64_t bytes, hipStream_t s);
int launch_probe_stream(int reads, int writes, int unroll, int nontemporal, int grid, void *dst, const void *src,
                        int64_t bytes, hipStream_t s);
int launch_kpm_moments(const double *dots, int64_t M, int32_t b, double *mu, hipStream_t s);
// dot[g * dot_b + j] = sum_t partials[(g * nb + j) * nparts + t] for the groups g requested
// in flags (yy, xy, xx), fixed summation order; batch > 1 handles consecutive partial
// blocks (stride 3 * nb * nparts, or part_stride) writing dot + k * dot_stride.
int launch_dot_finish(const double *partials, int32_t nparts, int32_t nb, uint32_t flags, double *dot,
                      int32_t dot_b, int64_t batch, int64_t dot_stride, hipStream_t s);
int launch_dot_finish_strided(const double *partials, int32_t nparts, int32_t nb, uint32_t flags, double *dot,
                              int32_t dot_b, int64_t batch, int64_t dot_stride, int64_t part_stride,
                              hipStream_t s);

// CG building blocks (cg.hip): FP64 scalars live on the device.
constexpr int kCgMaxGrid = 1024;  // workgroups of the reducing vector kernels
struct CgDev {
    double *rho;      // <r, r> per column (b)
    double *pq;       // <p, A p> per column (b)
    double *alpha;    // b
    double *beta;     // b
    double *thresh2;  // squared stopping threshold per column (b)
    int32_t *active;  // per column: 1 while not converged
};
unsigned cg_reduce_grid(int64_t n, int b);
// alpha and beta per column from the product's partials of <q, q> and <p, q> (q = A p)
int cg_launch_step(const double *prod_partials, int ntiles, int b, const CgDev &sc, hipStream_t s);
// r -= alpha q, x += alpha p, p = r + beta p in one pass with the partials of <r, r>, then rho
// and the column flags
int cg_launch_rp(int dt, void *R, const void *Q, void *P, void *X, int64_t n, int b, int64_t ld, const CgDev &sc,
                 double *partials, hipStream_t s);
int cg_launch_coldot(int dt, const void *U, const void *V, int64_t n, int b, int64_t ld, double *result,
                     double *partials, double *thresh2, int32_t *active, const double *ref, double f2,
                     hipStream_t s);
// P = R in the columns with colmask[j] != 0 (device flags)
int cg_launch_copy_cols(int dt, void *P, const void *R, int64_t n, int b, int64_t ld, const int32_t *colmask,
                        hipStream_t s);
int cg_launch_axpy_mixed(double *X, const float *D, int64_t n, int b, int64_t ld, hipStream_t s);

// Batched CG (cg.hip): K systems stored one after another in the block vectors.
struct BatchSeg {
    const int64_t *row_off;  // K + 1 row offsets (device)
    const int32_t *vblk;     // K + 1 workgroup offsets of the vector kernels (device)
    int32_t K, G;            // systems; workgroups of a vector launch (vblk[K])
    int64_t rows;            // rows of the whole batch (row_off[K])
};
struct BatchCg {
    double *rho, *alpha, *beta, *thresh2;  // K * b each, index m * b + j
    int32_t *active;                       // K * b column flags
    int32_t *sys_active;                   // K system flags (some column active)
    int64_t *iters;                        // K iteration counters
};
// alpha and beta of the iterating systems from the batched product's partials
int bcg_launch_step(const double *pparts, const int32_t *pblk, int K, int b, const BatchCg &sc, hipStream_t s);
// r -= alpha q, d += alpha p, p = r + beta p on the iterating systems' rows in one pass with
// the partials of <r, r>, then rho, the flags and the iteration counters
int bcg_launch_rp(int dt, void *R, const void *Q, void *P, void *D, int b, const BatchSeg &sg, const BatchCg &sc,
                  double *partials, hipStream_t s);
int bcg_launch_coldot(int dt, const void *U, const void *V, int b, const BatchSeg &sg, const int32_t *mask,
                      double *partials, double *result, double *thresh2, const double *ref, double f2,
                      hipStream_t s);
int bcg_launch_refresh_prep(int dt, double *X, void *D, double *R64, const double *Bv, int b, const BatchSeg &sg,
                            const int32_t *mask, hipStream_t s);
int bcg_launch_convert(int dt, void *R, const double *R64, int b, const BatchSeg &sg, const int32_t *mask,
                       double *partials, double *rho, double *thresh2, const double *ref, double f2, hipStream_t s);
// P = R in the columns with colmask[m * b + j] != 0
int bcg_launch_copy(int dt, void *P, const void *R, int b, const BatchSeg &sg, const int32_t *colmask,
                    hipStream_t s);
int launch_batch_dot_finish(const double *partials, const int32_t *blk, int K, int32_t nb, uint32_t flags,
                            double *dot, hipStream_t s);
int launch_batch_dot_finish_packed(const double *partials, const int32_t *blk, const int32_t *nbm,
                                   const int64_t *dot_off, int K, int32_t wmax, uint32_t flags, double *dot,
                                   hipStream_t s);

// The fused product of capi.cpp (no argument checks): y = alpha (A x - gamma x) + beta y,
// dots, chain; aug = false runs the plain product y = A x.
// partials_out == nullptr: the dots are summed into o.dot right away (workspace partials and
// a finishing kernel). Else the tile partials of the (single, b <= 64) slice are left in
// partials_out (3 * b * ntiles doubles) for the caller to reduce, and o.dot is not used.
// *nblocks_out (may be null) receives the number of partials per quantity (workgroups).
// ws_in: the reduction partials and lane scratch to use; nullptr takes the stream's workspace
// (allocated on the first call on a stream).
struct Workspace;
int aug_impl(const sell_mat *A, const sell_bv *X, sell_bv *Y, sell_bv *Z, const sell_spmv_opts &o, bool aug,
             hipStream_t s, double *partials_out = nullptr, int32_t *nblocks_out = nullptr,
             const Workspace *ws_in = nullptr);
// Checks the operands of sell_spmmv_aug and fills *o from opts (the defaults when null).
int check_aug_call(const sell_mat *A, const sell_bv *X, sell_bv *Y, sell_bv *Z, const sell_spmv_opts *opts,
                   sell_spmv_opts *o);
// Workgroups of one product launch: as many as the device holds at once (occupancy of the
// kernel times the compute units), at most the number of fine tiles.
// blocks_per_cu > 0 lowers the workgroups per compute unit to at most that many.
int32_t resident_grid(const void *kernel, int threads, int32_t ntiles, int32_t blocks_per_cu = 0);
// Columns per lane of the fixed-width product kernels: hint (1, 2 or 4, at most b) when
// given, else 4 for b >= 4 and b otherwise.
int choose_vpt(int vk, int b, int hint = 0);

// Lazily built device maps (row -> slot, CSR row pointers) and the SELL copy of A^T.
int ensure_update_maps(sell_mat *A, hipStream_t s);
int ensure_transpose(const sell_mat *A, hipStream_t s);
// Page lists and tile-local column indices for the LDS-staged product (stage.hip), over stage
// tiles of `chunks` consecutive chunks; rebuilt when a different tile size is asked for.
int ensure_stage(const sell_mat *A, int32_t chunks, hipStream_t s);
// The slot plan of a staged launch with nblk workgroups, unit stride (0: contiguous) and ns
// cache slots (stage.hip); rebuilt when any of them changes.
int ensure_stage_plan(const sell_mat *A, int32_t nblk, int32_t stride, int32_t ns, hipStream_t s);

// Value-gradient kernels (grad.hip).
int launch_grad_accum(const sell_mat *A, const void *G, int64_t ldg, const void *X, int64_t ldx, int vec_dt,
                      int32_t b, double alpha, double *dsell, hipStream_t s);
int launch_sell_to_csr(const sell_mat *A, const double *dsell, int accumulate, double *dval, hipStream_t s);
int launch_axpby(int vec_dt, int64_t n, int32_t b, int64_t ld, double alpha, const void *x, double beta, void *y,
                 hipStream_t s);
// dst[pos[p]] = convert(src[p]) for p < n, dst of storage type vdt
int launch_scatter_values(const double *src, const int64_t *pos, int64_t n, int vdt, void *dst, hipStream_t s);

// Device and pinned host allocations of the library (alloc.cpp): hipMalloc and friends with a
// count of live allocations and a test hook that makes the k-th next allocation fail.
hipError_t lib_malloc(void **p, size_t bytes);
hipError_t lib_malloc_async(void **p, size_t bytes, hipStream_t s);
hipError_t lib_host_malloc(void **p, size_t bytes, unsigned flags);
hipError_t lib_free(void *p);
hipError_t lib_free_async(void *p, hipStream_t s);
hipError_t lib_host_free(void *p);
template <class T>
hipError_t lib_malloc(T **p, size_t bytes) {
    return lib_malloc(reinterpret_cast<void **>(p), bytes);
}
template <class T>
hipError_t lib_malloc_async(T **p, size_t bytes, hipStream_t s) {
    return lib_malloc_async(reinterpret_cast<void **>(p), bytes, s);
}

// Argument helpers of the entry points (capi.cpp).
int check_device(const sell_mat *A);     // on the device and the current one
int validate_bv(const sell_bv *v);
int vec_kind(int vdt);                   // VecKind of a value type
int vec_dtype_for(int vdt);              // block-vector type for a value type
void bv_strides(const sell_bv *v, int64_t &rs, int64_t &cs);
char *elem_ptr(const sell_bv *v, int64_t i, int64_t j);
void base_args(ProdArgs &a, const sell_mat *A);  // matrix fields of a product launch

// Per-(device, stream) workspace for reductions.
struct Workspace {
    double *partials = nullptr;   // kMaxTiles * 3 * kMaxSliceCols doubles
    void *scratch = nullptr;      // write-only scratch of the product kernels (kScratchBytes)
};
constexpr size_t kScratchBytes = size_t(kBlock) * 64;
int get_workspace(hipStream_t s, Workspace **ws);
// Frees the workspace of a stream that is about to be destroyed (after its work has finished).
void drop_workspace(hipStream_t s);

}  // namespace sellcs
