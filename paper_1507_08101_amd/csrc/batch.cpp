// batch.cpp -- products over a batch of independent matrices in one kernel launch.
//
// The batch's block vectors hold the matrices' operands one after another: matrix m reads
// rows [col_off[m], col_off[m+1]) of X and writes rows [row_off[m], row_off[m+1]) of Y. One
// launch of the batched product kernel covers every matrix: sixteen waves of the device's resident
// workgroups are split over the matrices by their cost (stored entries plus rows) so that the
// busiest workgroup has as little work as possible, and each workgroup finds its matrix's launch arguments in a table in device memory by a binary
// search over the workgroup offsets. The tables are staged through pinned host memory into a
// few device slots; a call whose table equals one already on the device (the same operands
// and scalars, as in every iteration of a solver) uploads nothing, which keeps repeated calls
// free of copies and lets them be captured in a HIP graph.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <queue>
#include <utility>

#include "internal.h"
#include "log.h"

using namespace sellcs;

namespace sellcs {
const void *batch_kernel_f64(int b, int vpt, bool aug, bool fixed_ok, int ub, int ubw, uint32_t flags);
const void *batch_kernel_f32(int b, int vpt, bool aug, bool fixed_ok, int ub, int ubw, uint32_t flags);
const void *batch_kernel_bf16(int b, int vpt, bool aug, bool fixed_ok, int ub, int ubw, uint32_t flags);
const void *batch_mixed_kernel_f64(bool aug);
const void *batch_mixed_kernel_f32(bool aug);
const void *batch_mixed_kernel_bf16(bool aug);
}  // namespace sellcs

namespace {

#define HIPCHK(x)                                                                             \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess) return e_ == hipErrorOutOfMemory ? SELL_ERR_OOM : SELL_ERR_HIP; \
    } while (0)

constexpr int kRing = 4;            // table slots shared by all calls, reused round robin
constexpr int kSlots = kRing + 1;   // plus one reserved for a solver's repeated product

bool fixed_width(int b) { return b == 1 || b == 2 || b == 4 || b == 8 || b == 16 || b == 32; }

bool vec_ok(const void *p, int64_t rs, int64_t cs, int esize, int align) {
    return cs == 1 && (reinterpret_cast<uintptr_t>(p) % align) == 0 && ((rs * esize) % align) == 0;
}

}  // namespace

struct sell_batch {
    std::vector<const sell_mat *> mats;
    int32_t K = 0;
    int device = -1;
    int vdt = SELL_F64;
    int64_t rows = 0, cols = 0;
    std::vector<int64_t> row_off, col_off;  // K + 1
    std::vector<double> cost;               // per matrix
    int64_t total_tiles = 0;
    // table slots: K ProdArgs followed by K + 1 int32 workgroup offsets
    size_t table_bytes = 0;
    void *d_slot[kSlots] = {};
    void *h_slot[kSlots] = {};  // pinned staging copies (also the record of the slot content)
    hipEvent_t ev[kSlots] = {};
    bool valid[kSlots] = {};
    int next = 0;
    std::vector<uint8_t> stage;
    double *partials = nullptr;
    size_t partials_cap = 0;  // doubles
    int64_t *d_row_off = nullptr;  // device copy of row_off (for the batched solvers)
    int32_t *d_vblk = nullptr;     // vector-kernel workgroup offsets (for the batched solvers)
    int32_t vgrid = 0;
    int32_t vpt_hint = 0, bpc_hint = 0;  // launch parameters shared by all matrices (else 0)
    int32_t batch_len = 8;               // index batch length shared by all matrices (else 8)
    int32_t batch_len_wide = 8;          // the same for the kernels gathering 32 bytes per lane
    std::map<int32_t, std::vector<int32_t>> blk_cache;  // workgroup offsets per resident grid size
    // block widths of the matrices for packed operands (empty: not set)
    std::vector<int32_t> widths;
    std::vector<int64_t> xoff, yoff;                       // element offsets of the packed blocks
    int64_t x_elems = 0, y_elems = 0, sum_w = 0;
    int32_t wmax = 0;
    int32_t *d_widths = nullptr;
    int64_t *d_dotoff = nullptr;                           // sum of the earlier widths, per matrix
    std::vector<int32_t> porder;                           // launch-table position -> matrix, by width
    std::vector<double> cost_w;                            // per matrix, at its own width
    std::map<int32_t, std::vector<int32_t>> blk_cache_w;   // offsets for the widths' costs
};

namespace sellcs {

void batch_free(sell_batch *B) {
    for (int i = 0; i < kSlots; ++i) {
        if (B->ev[i]) (void)hipEventSynchronize(B->ev[i]);
        if (B->ev[i]) (void)hipEventDestroy(B->ev[i]);
        if (B->d_slot[i]) (void)lib_free(B->d_slot[i]);
        if (B->h_slot[i]) (void)lib_host_free(B->h_slot[i]);
    }
    if (B->partials) (void)lib_free(B->partials);
    if (B->d_row_off) (void)lib_free(B->d_row_off);
    if (B->d_vblk) (void)lib_free(B->d_vblk);
    if (B->d_widths) (void)lib_free(B->d_widths);
    if (B->d_dotoff) (void)lib_free(B->d_dotoff);
}

// True when the matrices have widths of their own that differ from the operands' width b.
bool batch_ragged(const sell_batch *B, int b) {
    for (int32_t w : B->widths)
        if (w != b) return true;
    return false;
}

const sell_mat *batch_matrix(const sell_batch *B, int m) { return B->mats[size_t(m)]; }
int32_t batch_count(const sell_batch *B) { return B->K; }
int64_t batch_rows(const sell_batch *B) { return B->rows; }
int batch_vdt(const sell_batch *B) { return B->vdt; }

// Segment description of the batch for the vector kernels of the batched solvers.
BatchSeg batch_seg(const sell_batch *B) {
    BatchSeg sg;
    sg.row_off = B->d_row_off;
    sg.vblk = B->d_vblk;
    sg.K = B->K;
    sg.G = B->vgrid;
    sg.rows = B->rows;
    return sg;
}

// Splits G0 workgroups over K items so that the largest work per workgroup is as small as
// possible: one for every item with work (cap > 0), then one at a time to the item whose work
// per workgroup is largest (ties to the lower index), never more than cap. A launch takes as long
// as its busiest workgroup, so this is the split that finishes first (a proportional split
// rounds an item of 1.4 workgroups' worth down to one and leaves that workgroup 40 % over).
// blk receives the K + 1 offsets; the total exceeds G0 only when more items have work than G0.
void apportion(const std::vector<double> &w, const std::vector<int64_t> &cap, int32_t G0,
               std::vector<int32_t> &blk) {
    const size_t K = w.size();
    std::vector<int64_t> n(K, 0);
    std::priority_queue<std::pair<double, int64_t>> q;  // (work per workgroup, -index)
    int64_t sum = 0;
    for (size_t m = 0; m < K; ++m) {
        if (cap[m] <= 0) continue;
        n[m] = 1;
        ++sum;
        if (cap[m] > 1) q.emplace(w[m], -int64_t(m));
    }
    while (sum < G0 && !q.empty()) {
        const size_t m = size_t(-q.top().second);
        q.pop();
        ++n[m];
        ++sum;
        if (n[m] < cap[m]) q.emplace(w[m] / double(n[m]), -int64_t(m));
    }
    blk.assign(K + 1, 0);
    for (size_t m = 0; m < K; ++m) blk[m + 1] = blk[m] + int32_t(n[m]);
}

// Workgroups of the product launches per matrix: weights = cost, cap = fine tiles; matrices
// with host_active[m] == 0 get none (host_active may be null: all matrices).
void apportion_products(const sell_batch *B, int32_t G0, const int32_t *host_active, std::vector<int32_t> &blk,
                        bool ragged = false) {
    std::vector<int64_t> cap(static_cast<size_t>(B->K));
    for (int m = 0; m < B->K; ++m)
        cap[size_t(m)] = (host_active && !host_active[m]) ? 0 : B->mats[size_t(m)]->ntiles;
    apportion(ragged ? B->cost_w : B->cost, cap, G0, blk);
}

namespace {

// Workgroups of a product launch with kernel kern: 16 waves of the resident grid by default. A
// finer split than one wave balances uneven matrices better, since workgroups that finish early
// take the next ones (64 Laplacians of edges 20..100 at b = 8: 1.42 ms with 16 waves, 1.68 ms
// with 2, 1.83 ms with 1; mixed widths 1..32: 2.85 ms against 4.06 ms with 2).
int32_t product_grid(const sell_batch *B, const void *kern) {
    static const int32_t waves = [] {
        const char *e = std::getenv("SELLCS_BATCH_WAVES");
        const int v = e ? std::atoi(e) : 16;
        return int32_t(v >= 1 && v <= 32 ? v : 16);
    }();
    return waves * resident_grid(kern, kBlock, int32_t(std::min<int64_t>(B->total_tiles, 1 << 30)), B->bpc_hint);
}

// Room for 3 * kMaxSliceCols partials per workgroup of any split of this grid, so that later
// calls (possibly captured in a graph) never move the buffer.
int ensure_partials(sell_batch *B, int32_t G, int32_t G0) {
    const size_t need = size_t(3) * kMaxSliceCols * size_t(std::max<int64_t>(std::max(G, G0), B->K));
    if (need <= B->partials_cap) return SELL_OK;
    // grows outside any steady state (the first call of a shape)
    if (B->partials) HIPCHK(lib_free(B->partials));
    B->partials = nullptr;
    B->partials_cap = 0;
    HIPCHK(lib_malloc(&B->partials, need * sizeof(double)));
    B->partials_cap = need;
    return SELL_OK;
}

// Appends the workgroup offsets to the staged table (K ProdArgs already in B->stage) and finds
// the table on the device, else uploads it (into the reserved slot, or the next ring slot).
int place_table(sell_batch *B, const std::vector<int32_t> &blk, bool reserved, hipStream_t s,
                const ProdArgs **d_tab, const int32_t **d_blk) {
    const int K = B->K;
    std::memcpy(B->stage.data() + sizeof(ProdArgs) * size_t(K), blk.data(), sizeof(int32_t) * (size_t(K) + 1));
    int slot = -1;
    if (reserved) {
        if (B->valid[kRing] && std::memcmp(B->h_slot[kRing], B->stage.data(), B->table_bytes) == 0) slot = kRing;
    } else {
        for (int i = 0; i < kRing && slot < 0; ++i)
            if (B->valid[i] && std::memcmp(B->h_slot[i], B->stage.data(), B->table_bytes) == 0) slot = i;
    }
    if (slot < 0) {
        if (reserved) {
            slot = kRing;
        } else {
            slot = B->next;
            B->next = (B->next + 1) % kRing;
        }
        if (B->valid[slot]) HIPCHK(hipEventSynchronize(B->ev[slot]));  // its last upload has been read
        B->valid[slot] = false;
        std::memcpy(B->h_slot[slot], B->stage.data(), B->table_bytes);
        HIPCHK(hipMemcpyAsync(B->d_slot[slot], B->h_slot[slot], B->table_bytes, hipMemcpyHostToDevice, s));
        HIPCHK(hipEventRecord(B->ev[slot], s));
        B->valid[slot] = true;
    }
    *d_tab = static_cast<const ProdArgs *>(B->d_slot[slot]);
    *d_blk = reinterpret_cast<const int32_t *>(static_cast<const char *>(B->d_slot[slot]) + sizeof(ProdArgs) * size_t(K));
    return SELL_OK;
}

// The epilogue fields of a launch-table entry (nb columns of the shifts).
void set_epilogue(ProdArgs &a, const sell_spmv_opts &o) {
    a.flags = o.flags;
    a.alpha = o.alpha;
    a.beta = o.beta;
    a.delta = o.delta;
    a.eta = o.eta;
    a.gamma_s = o.gamma;
    if (o.flags & SELL_SPMV_VSHIFT) {
        a.has_gamma_v = 1;
        for (int j = 0; j < a.nb; ++j) a.gamma_v[j] = o.gamma_v[j];
    }
}

}  // namespace

// The batched product (no argument checks): y_m = alpha (A_m x_m - gamma x_m) + beta y_m with
// dots and chain for every matrix m, skipping matrices with active[m] == 0 (device flags read
// by the kernel; may be null). host_active (K host flags, may be null) restricts the launch to
// the flagged matrices: the others get no workgroups and are not touched, and the resident
// grid is split over the flagged ones only. Dot partials stay in the batch's buffer;
// *out_blk / *out_partials (may be null) receive the device workgroup offsets and the partials.
// finish: sum the dots into o.dot (3 b doubles per matrix; those of unlaunched matrices are
// left as they are). reserved: keep the launch table in the batch's reserved slot, which only
// other reserved calls replace (a solver's repeated product, whose table a captured graph
// refers to, is not evicted by its other products).
int batch_aug_impl(sell_batch *B, const sell_bv *X, sell_bv *Y, sell_bv *Z, const sell_spmv_opts &o, bool aug,
                   const int32_t *active, const int32_t *host_active, bool finish, hipStream_t s,
                   const int32_t **out_blk, const double **out_partials, bool reserved) {
    const int b = X->ncols;
    const int K = B->K;
    if (batch_ragged(B, b)) return SELL_ERR_UNSUPPORTED;  // mixed widths take packed operands
    Workspace *ws = nullptr;
    int rc = get_workspace(s, &ws);
    if (rc) return rc;
    const int vk = vec_kind(B->vdt);
    const int esize = vk == VK_F64F64 ? 8 : 4;
    const int vpt = choose_vpt(vk, b, B->vpt_hint);
    const int align = vpt * esize < 16 ? vpt * esize : 16;
    int64_t xrs, xcs, yrs, ycs, zrs = 0, zcs = 0;
    bv_strides(X, xrs, xcs);
    bv_strides(Y, yrs, ycs);
    const bool chain = aug && (o.flags & SELL_SPMV_CHAIN);
    if (chain) bv_strides(Z, zrs, zcs);
    bool fixed_ok = fixed_width(b) && vec_ok(X->ptr, xrs, xcs, esize, align) && vec_ok(Y->ptr, yrs, ycs, esize, align);
    if (chain) fixed_ok = fixed_ok && vec_ok(Z->ptr, zrs, zcs, esize, align);
    if (!fixed_ok)
        log_warn_once(kWarnBatchGeneral,
                      "batched product with block width %d and these block vectors (a width other than 1, 2, "
                      "4, 8, 16, 32, or rows that are not row-major and %d-byte aligned): the run-time-width "
                      "kernel runs",
                      b, align);
    const int ub = B->batch_len, ubw = B->batch_len_wide;
    const uint32_t kflags = aug ? o.flags : 0u;  // every matrix of the launch has these flags
    const void *kern = vk == VK_F64F64   ? batch_kernel_f64(b, vpt, aug, fixed_ok, ub, ubw, kflags)
                       : vk == VK_F32F32 ? batch_kernel_f32(b, vpt, aug, fixed_ok, ub, ubw, kflags)
                                         : batch_kernel_bf16(b, vpt, aug, fixed_ok, ub, ubw, kflags);
    // workgroups per matrix: waves of the resident grid split so that the busiest workgroup
    // has as little work as possible
    const int32_t G0 = product_grid(B, kern);
    std::vector<int32_t> sub_blk;
    const std::vector<int32_t> *pblk_h = nullptr;
    if (host_active) {
        apportion_products(B, G0, host_active, sub_blk);
        pblk_h = &sub_blk;
    } else {
        auto hit = B->blk_cache.find(G0);
        if (hit == B->blk_cache.end()) {
            std::vector<int32_t> v;
            apportion_products(B, G0, nullptr, v);
            hit = B->blk_cache.emplace(G0, std::move(v)).first;
        }
        pblk_h = &hit->second;
    }
    const std::vector<int32_t> &blk = *pblk_h;
    const int32_t G = blk[size_t(K)];
    const bool dots = aug && (o.flags & SELL_SPMV_DOTS);
    if (dots && (rc = ensure_partials(B, G, G0))) return rc;
    // the table
    B->stage.assign(B->table_bytes, 0);
    ProdArgs *tab = reinterpret_cast<ProdArgs *>(B->stage.data());
    for (int m = 0; m < K; ++m) {
        const sell_mat *A = B->mats[size_t(m)];
        ProdArgs a;
        base_args(a, A);
        a.nb = b;
        a.nblocks = blk[size_t(m) + 1] - blk[size_t(m)];
        a.tile_stride = 0;
        a.stage = 0;
        a.xrs = xrs;
        a.xcs = xcs;
        a.yrs = yrs;
        a.ycs = ycs;
        a.X = elem_ptr(X, B->col_off[size_t(m)], 0);
        a.Y = elem_ptr(Y, B->row_off[size_t(m)], 0);
        a.scratch = ws->scratch;
        if (chain) {
            a.zrs = zrs;
            a.zcs = zcs;
            a.Z = elem_ptr(Z, B->row_off[size_t(m)], 0);
        }
        if (aug) {
            set_epilogue(a, o);
            if (dots) a.partials = B->partials + size_t(3) * b * blk[size_t(m)];
        }
        std::memcpy(&tab[m], &a, sizeof(ProdArgs));
    }
    const ProdArgs *d_tab = nullptr;
    const int32_t *d_blk = nullptr;
    if ((rc = place_table(B, blk, reserved, s, &d_tab, &d_blk))) return rc;
    if (out_blk) *out_blk = d_blk;
    if (out_partials) *out_partials = B->partials;
    if (G > 0) {
        int vl_log2 = 0;
        if (!fixed_ok)
            while ((1 << vl_log2) < b) ++vl_log2;
        int Karg = K;
        void *args[] = {&d_tab, &d_blk, &Karg, &active, &vl_log2};
        HIPCHK(hipLaunchKernel(kern, dim3(unsigned(G)), dim3(kBlock), args, 0, s));
    }
    if (dots && finish) {
        if (G == 0) {
            for (int m = 0; m < K; ++m)
                if ((rc = launch_fill(o.dot + size_t(m) * 3 * b, SELL_F64, 1, 3 * b, 3 * b, 1, 0.0, s))) return rc;
            return SELL_OK;
        }
        if (host_active) {
            // only the launched matrices have partials (a matrix without rows: zero dots)
            for (int m = 0; m < K; ++m) {
                if (!host_active[m]) continue;
                const int32_t np = blk[size_t(m) + 1] - blk[size_t(m)];
                double *dm = o.dot + size_t(m) * 3 * b;
                rc = np > 0 ? launch_dot_finish(B->partials + size_t(3) * b * blk[size_t(m)], np, b, o.flags, dm, b,
                                                1, 0, s)
                            : launch_fill(dm, SELL_F64, 1, 3 * b, 3 * b, 1, 0.0, s);
                if (rc) return rc;
            }
            return SELL_OK;
        }
        if ((rc = launch_batch_dot_finish(B->partials, d_blk, K, b, o.flags, o.dot, s))) return rc;
    }
    return SELL_OK;
}

// The batched product over packed operands of per-matrix widths (no argument checks):
// matrix m's X block starts at element xoff[m] of X (ncols_m x w_m, row-major, ld = w_m), its
// Y and Z blocks at yoff[m]; its dots land packed at o.dot + 3 dotoff[m]. One launch of the
// mixed-width kernel; the launch table lists the matrices by width, and the workgroups are
// split by each matrix's cost at its own width.
int batch_aug_packed_impl(sell_batch *B, const void *X, void *Y, void *Z, const sell_spmv_opts &o, bool aug,
                          hipStream_t s) {
    const int K = B->K;
    Workspace *ws = nullptr;
    int rc = get_workspace(s, &ws);
    if (rc) return rc;
    const int vk = vec_kind(B->vdt);
    const int esize = vk == VK_F64F64 ? 8 : 4;
    const bool chain = aug && (o.flags & SELL_SPMV_CHAIN);
    const void *kern = vk == VK_F64F64   ? batch_mixed_kernel_f64(aug)
                       : vk == VK_F32F32 ? batch_mixed_kernel_f32(aug)
                                         : batch_mixed_kernel_bf16(aug);
    const int32_t G0 = product_grid(B, kern);
    auto hit = B->blk_cache_w.find(G0);
    if (hit == B->blk_cache_w.end()) {
        // workgroups per table position (matrices in width order)
        std::vector<double> w(static_cast<size_t>(K));
        std::vector<int64_t> cap(static_cast<size_t>(K));
        for (int p = 0; p < K; ++p) {
            const int32_t m = B->porder[size_t(p)];
            w[size_t(p)] = B->cost_w[size_t(m)];
            cap[size_t(p)] = B->mats[size_t(m)]->ntiles;
        }
        std::vector<int32_t> v;
        apportion(w, cap, G0, v);
        hit = B->blk_cache_w.emplace(G0, std::move(v)).first;
    }
    const std::vector<int32_t> &blk = hit->second;
    const int32_t G = blk[size_t(K)];
    const bool dots = aug && (o.flags & SELL_SPMV_DOTS);
    if (dots && (rc = ensure_partials(B, G, G0))) return rc;
    const char *xb = static_cast<const char *>(X);
    char *yb = static_cast<char *>(Y), *zb = static_cast<char *>(Z);
    B->stage.assign(B->table_bytes, 0);
    ProdArgs *tab = reinterpret_cast<ProdArgs *>(B->stage.data());
    for (int p = 0; p < K; ++p) {
        const int32_t m = B->porder[size_t(p)];
        const sell_mat *A = B->mats[size_t(m)];
        const int w = B->widths[size_t(m)];
        ProdArgs a;
        base_args(a, A);
        a.nb = w;
        a.nblocks = blk[size_t(p) + 1] - blk[size_t(p)];
        a.tile_stride = 0;
        a.stage = 0;
        a.X = xb + B->xoff[size_t(m)] * esize;
        a.Y = yb + B->yoff[size_t(m)] * esize;
        a.xrs = a.yrs = w;
        a.xcs = a.ycs = 1;
        if (chain) {
            a.Z = zb + B->yoff[size_t(m)] * esize;
            a.zrs = w;
            a.zcs = 1;
        }
        // the compiled body needs rows aligned to its vector accesses
        const int vpt = w >= 4 ? 4 : w;
        const int al = vpt * esize < 16 ? vpt * esize : 16;
        bool vec = fixed_width(w) && vec_ok(a.X, w, 1, esize, al) && vec_ok(a.Y, w, 1, esize, al);
        if (chain) vec = vec && vec_ok(a.Z, w, 1, esize, al);
        a.runtime_width = vec ? 0 : 1;
        a.scratch = ws->scratch;
        if (aug) {
            set_epilogue(a, o);
            if (dots) a.partials = B->partials + size_t(3) * B->wmax * blk[size_t(p)];
        }
        std::memcpy(&tab[p], &a, sizeof(ProdArgs));
    }
    const ProdArgs *d_tab = nullptr;
    const int32_t *d_blk = nullptr;
    if ((rc = place_table(B, blk, false, s, &d_tab, &d_blk))) return rc;
    if (G > 0) {
        int vl_log2 = 0;  // unused by the mixed-width kernel
        int Karg = K;
        const int32_t *active = nullptr;
        void *args[] = {&d_tab, &d_blk, &Karg, &active, &vl_log2};
        HIPCHK(hipLaunchKernel(kern, dim3(unsigned(G)), dim3(kBlock), args, 0, s));
    }
    if (dots) {
        if (G == 0) return launch_fill(o.dot, SELL_F64, 1, int32_t(3 * B->sum_w), 3 * B->sum_w, 1, 0.0, s);
        return launch_batch_dot_finish_packed(B->partials, d_blk, B->d_widths, B->d_dotoff, K, B->wmax, o.flags,
                                              o.dot, s);
    }
    return SELL_OK;
}

}  // namespace sellcs

extern "C" {

int sell_batch_create(sell_mat *const *mats, int32_t count, sell_batch **out) {
    if (!out) return SELL_ERR_ARG;
    *out = nullptr;
    if (!mats || count < 1) return SELL_ERR_ARG;
    int cur = -1;
    HIPCHK(hipGetDevice(&cur));
    for (int32_t m = 0; m < count; ++m) {
        int rc = check_device(mats[m]);
        if (rc) return rc;
        if (mats[m]->h.vdt != mats[0]->h.vdt) return SELL_ERR_DTYPE;
    }
    sell_batch *B = new (std::nothrow) sell_batch();
    if (!B) return SELL_ERR_OOM;
    int rc = SELL_OK;
    try {
        B->K = count;
        B->device = cur;
        B->vdt = mats[0]->h.vdt;
        B->mats.assign(mats, mats + count);
        B->row_off.assign(size_t(count) + 1, 0);
        B->col_off.assign(size_t(count) + 1, 0);
        B->cost.assign(size_t(count), 0.0);
        for (int32_t m = 0; m < count; ++m) {
            const HostSell &h = mats[m]->h;
            B->row_off[size_t(m) + 1] = B->row_off[size_t(m)] + h.nrows;
            B->col_off[size_t(m) + 1] = B->col_off[size_t(m)] + h.ncols;
            B->cost[size_t(m)] = double(h.stored) + double(h.nrows);
            B->total_tiles += std::max(0, mats[m]->ntiles);
        }
        B->rows = B->row_off[size_t(count)];
        // launch parameters chosen for the matrices apply to the batch when they all agree
        B->vpt_hint = mats[0]->vpt_hint;
        B->bpc_hint = mats[0]->bpc_hint;
        for (int32_t m = 1; m < count; ++m) {
            if (mats[m]->vpt_hint != B->vpt_hint) B->vpt_hint = 0;
            if (mats[m]->bpc_hint != B->bpc_hint) B->bpc_hint = 0;
        }
        // one kernel serves every matrix of a launch: their common index batch length, else 8
        auto blen = [](const sell_mat *M) { return M->batch_hint > 0 ? M->batch_hint : M->h.batch; };
        auto blenw = [](const sell_mat *M) { return M->batch_hint > 0 ? M->batch_hint : M->h.batch_wide; };
        B->batch_len = blen(mats[0]);
        B->batch_len_wide = blenw(mats[0]);
        for (int32_t m = 1; m < count; ++m) {
            if (blen(mats[m]) != B->batch_len) B->batch_len = 8;
            if (blenw(mats[m]) != B->batch_len_wide) B->batch_len_wide = 8;
        }
        B->cols = B->col_off[size_t(count)];
        B->table_bytes = sizeof(ProdArgs) * size_t(count) + sizeof(int32_t) * (size_t(count) + 1);
    } catch (const std::bad_alloc &) {
        delete B;
        return SELL_ERR_OOM;
    }
    auto fail = [&](hipError_t e) {
        batch_free(B);
        delete B;
        return e == hipErrorOutOfMemory ? SELL_ERR_OOM : SELL_ERR_HIP;
    };
    hipError_t e;
    for (int i = 0; i < kSlots; ++i) {
        if ((e = lib_malloc(&B->d_slot[i], B->table_bytes)) != hipSuccess) return fail(e);
        if ((e = lib_host_malloc(&B->h_slot[i], B->table_bytes, hipHostMallocDefault)) != hipSuccess) return fail(e);
        if ((e = hipEventCreateWithFlags(&B->ev[i], hipEventDisableTiming)) != hipSuccess) return fail(e);
    }
    // vector-kernel workgroups for the batched solvers: 2 * kCgMaxGrid in total, split by the
    // rows (at least one per non-empty system, a few rows per workgroup)
    {
        const int32_t Gv = 2 * kCgMaxGrid;
        std::vector<int32_t> vblk;
        std::vector<double> w(static_cast<size_t>(count));
        std::vector<int64_t> cap(static_cast<size_t>(count));
        for (int32_t m = 0; m < count; ++m) {
            const int64_t n = B->row_off[size_t(m) + 1] - B->row_off[size_t(m)];
            w[size_t(m)] = double(n);
            cap[size_t(m)] = n > 0 ? std::max<int64_t>(1, (n + 3) / 4) : 0;
        }
        apportion(w, cap, Gv, vblk);
        B->vgrid = vblk[size_t(count)];
        if ((e = lib_malloc(&B->d_row_off, sizeof(int64_t) * (size_t(count) + 1))) != hipSuccess) return fail(e);
        if ((e = lib_malloc(&B->d_vblk, sizeof(int32_t) * (size_t(count) + 1))) != hipSuccess) return fail(e);
        if ((e = hipMemcpy(B->d_row_off, B->row_off.data(), sizeof(int64_t) * (size_t(count) + 1),
                           hipMemcpyHostToDevice)) != hipSuccess)
            return fail(e);
        if ((e = hipMemcpy(B->d_vblk, vblk.data(), sizeof(int32_t) * (size_t(count) + 1), hipMemcpyHostToDevice)) !=
            hipSuccess)
            return fail(e);
    }
    (void)rc;
    *out = B;
    return SELL_OK;
}

int sell_batch_destroy(sell_batch *B) {
    if (!B) return SELL_OK;
    batch_free(B);
    delete B;
    return SELL_OK;
}

int sell_batch_info(const sell_batch *B, int32_t *count, int64_t *rows, int64_t *cols) {
    if (!B) return SELL_ERR_ARG;
    if (count) *count = B->K;
    if (rows) *rows = B->rows;
    if (cols) *cols = B->cols;
    return SELL_OK;
}

int sell_batch_set_widths(sell_batch *B, const int32_t *widths) {
    if (!B) return SELL_ERR_ARG;
    int cur = -1;
    HIPCHK(hipGetDevice(&cur));
    if (cur != B->device) return SELL_ERR_STATE;
    if (widths)
        for (int32_t m = 0; m < B->K; ++m)
            if (widths[m] < 1 || widths[m] > kMaxSliceCols) return SELL_ERR_ARG;
    // earlier launches may still read the device copies of the widths and offsets
    HIPCHK(hipDeviceSynchronize());
    if (!widths) {
        B->widths.clear();
        B->porder.clear();
        B->cost_w.clear();
        B->xoff.clear();
        B->yoff.clear();
        B->x_elems = B->y_elems = B->sum_w = 0;
        B->wmax = 0;
        B->blk_cache_w.clear();
        return SELL_OK;
    }
    // everything is computed aside and published at the end, so that a failure leaves the batch
    // as it was (or, after a failed copy to the device, without widths)
    if (!B->d_widths) HIPCHK(lib_malloc(&B->d_widths, sizeof(int32_t) * size_t(B->K)));
    if (!B->d_dotoff) HIPCHK(lib_malloc(&B->d_dotoff, sizeof(int64_t) * size_t(B->K)));
    const size_t K = size_t(B->K);
    std::vector<int32_t> wv, porder, w_ord;
    std::vector<int64_t> xoff, yoff, dotoff, off_ord;
    std::vector<double> cost;
    int64_t sum_w = 0;
    int32_t wmax = 0;
    try {
        wv.assign(widths, widths + K);
        xoff.assign(K + 1, 0);
        yoff.assign(K + 1, 0);
        dotoff.assign(K, 0);
        cost.assign(K, 0.0);
        // cost at the matrix's own width: its stored entries, the rows of X they gather (weighted
        // 0.7: mostly served by the caches; the factor reproduces the measured ratio of width-32
        // to width-1 batched products on 7-point Laplacians, 13x), and the rows of X and Y
        const double vb = B->vdt == SELL_F64 ? 8.0 : B->vdt == SELL_F32 ? 4.0 : 2.0;
        const double eb = B->vdt == SELL_F64 ? 8.0 : 4.0;
        for (size_t m = 0; m < K; ++m) {
            const HostSell &h = B->mats[m]->h;
            const int64_t w = widths[m];
            xoff[m + 1] = xoff[m] + h.ncols * w;
            yoff[m + 1] = yoff[m] + h.nrows * w;
            dotoff[m] = sum_w;
            sum_w += w;
            wmax = std::max<int32_t>(wmax, int32_t(w));
            cost[m] = double(h.stored) * (vb + 4.0 + 0.7 * double(w) * eb) + double(h.nrows + h.ncols) * double(w) * eb;
        }
        // the launch table lists the matrices by width (stable), so that the contiguous ranges
        // of workgroups that the XCDs receive hold matrices of one width where possible
        porder.resize(K);
        for (size_t m = 0; m < K; ++m) porder[m] = int32_t(m);
        std::stable_sort(porder.begin(), porder.end(), [&](int32_t x, int32_t y) { return widths[x] < widths[y]; });
        w_ord.resize(K);
        off_ord.resize(K);
        for (size_t p = 0; p < K; ++p) {
            w_ord[p] = widths[porder[p]];
            off_ord[p] = dotoff[size_t(porder[p])];
        }
    } catch (const std::bad_alloc &) {
        return SELL_ERR_OOM;
    }
    if (hipMemcpy(B->d_widths, w_ord.data(), sizeof(int32_t) * K, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(B->d_dotoff, off_ord.data(), sizeof(int64_t) * K, hipMemcpyHostToDevice) != hipSuccess) {
        B->widths.clear();  // the device copies may be stale: the batch has no widths now
        B->porder.clear();
        B->blk_cache_w.clear();
        return SELL_ERR_HIP;
    }
    B->widths.swap(wv);
    B->porder.swap(porder);
    B->xoff.swap(xoff);
    B->yoff.swap(yoff);
    B->cost_w.swap(cost);
    B->x_elems = B->xoff[K];
    B->y_elems = B->yoff[K];
    B->sum_w = sum_w;
    B->wmax = wmax;
    B->blk_cache_w.clear();
    return SELL_OK;
}

int sell_batch_packed_sizes(const sell_batch *B, int64_t *x_elems, int64_t *y_elems, int64_t *dots) {
    if (!B) return SELL_ERR_ARG;
    if (x_elems) *x_elems = B->x_elems;
    if (y_elems) *y_elems = B->y_elems;
    if (dots) *dots = 3 * B->sum_w;
    return SELL_OK;
}

int sell_batch_spmmv_aug_packed(sell_batch *B, const void *X, void *Y, void *Z, const sell_spmv_opts *opts,
                                void *stream) {
    if (!B) return SELL_ERR_ARG;
    int cur = -1;
    HIPCHK(hipGetDevice(&cur));
    if (cur != B->device) return SELL_ERR_STATE;
    if (B->widths.empty()) return SELL_ERR_STATE;
    const size_t esize = B->vdt == SELL_F64 ? 8 : 4;
    if ((B->x_elems > 0 && !X) || (B->y_elems > 0 && !Y)) return SELL_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Y)) % esize) return SELL_ERR_ARG;
    sell_spmv_opts o = SELL_SPMV_OPTS_INIT;
    if (opts) o = *opts;
    if (o.flags & ~0xFFu) return SELL_ERR_ARG;
    const uint32_t sq = SELL_SPMV_SHIFT | SELL_SPMV_VSHIFT | SELL_SPMV_DOT_XY | SELL_SPMV_DOT_XX;
    if (o.flags & sq)
        for (int m = 0; m < B->K; ++m)
            if (B->mats[size_t(m)]->h.nrows != B->mats[size_t(m)]->h.ncols) return SELL_ERR_SHAPE;
    if ((o.flags & SELL_SPMV_VSHIFT) && !o.gamma_v) return SELL_ERR_ARG;
    if ((o.flags & SELL_SPMV_DOTS) && !o.dot) return SELL_ERR_ARG;
    if (X == Y && B->y_elems > 0) return SELL_ERR_ARG;
    if (o.flags & SELL_SPMV_CHAIN) {
        if (B->y_elems > 0 && !Z) return SELL_ERR_ARG;
        if (reinterpret_cast<uintptr_t>(Z) % esize) return SELL_ERR_ARG;
        if (Z == Y && B->y_elems > 0) return SELL_ERR_ARG;
    }
    const bool aug = o.flags != 0;
    try {
        return batch_aug_packed_impl(B, X, Y, Z, o, aug, static_cast<hipStream_t>(stream));
    } catch (const std::bad_alloc &) {
        return SELL_ERR_OOM;
    }
}

int sell_batch_spmmv_aug(sell_batch *B, const sell_bv *X, sell_bv *Y, sell_bv *Z, const sell_spmv_opts *opts,
                         void *stream) {
    if (!B) return SELL_ERR_ARG;
    int cur = -1;
    HIPCHK(hipGetDevice(&cur));
    if (cur != B->device) return SELL_ERR_STATE;
    int rc;
    if ((rc = validate_bv(X)) || (rc = validate_bv(Y))) return rc;
    const int vdt = vec_dtype_for(B->vdt);
    if (X->dt != vdt || Y->dt != vdt) return SELL_ERR_DTYPE;
    if (X->ncols != Y->ncols || X->ncols < 1) return SELL_ERR_SHAPE;
    if (X->ncols > kMaxSliceCols) return SELL_ERR_UNSUPPORTED;
    if (X->nrows != B->cols || Y->nrows != B->rows) return SELL_ERR_SHAPE;
    if (batch_ragged(B, X->ncols)) return SELL_ERR_UNSUPPORTED;  // mixed widths take packed operands
    sell_spmv_opts o = SELL_SPMV_OPTS_INIT;
    if (opts) o = *opts;
    if (o.flags & ~0xFFu) return SELL_ERR_ARG;
    const uint32_t sq = SELL_SPMV_SHIFT | SELL_SPMV_VSHIFT | SELL_SPMV_DOT_XY | SELL_SPMV_DOT_XX;
    if (o.flags & sq)
        for (int m = 0; m < B->K; ++m)
            if (B->mats[size_t(m)]->h.nrows != B->mats[size_t(m)]->h.ncols) return SELL_ERR_SHAPE;
    if ((o.flags & SELL_SPMV_VSHIFT) && !o.gamma_v) return SELL_ERR_ARG;
    if ((o.flags & SELL_SPMV_DOTS) && !o.dot) return SELL_ERR_ARG;
    if (X->ptr == Y->ptr && B->rows > 0) return SELL_ERR_ARG;
    if (o.flags & SELL_SPMV_CHAIN) {
        if ((rc = validate_bv(Z))) return rc;
        if (Z->dt != Y->dt) return SELL_ERR_DTYPE;
        if (Z->nrows != Y->nrows || Z->ncols != Y->ncols) return SELL_ERR_SHAPE;
        if (Z->ptr == Y->ptr && B->rows > 0) return SELL_ERR_ARG;
    }
    const bool aug = o.flags != 0;
    try {
        return batch_aug_impl(B, X, Y, Z, o, aug, nullptr, nullptr, true, static_cast<hipStream_t>(stream), nullptr,
                              nullptr, false);
    } catch (const std::bad_alloc &) {
        return SELL_ERR_OOM;
    }
}

}  // extern "C"
