// capi.cpp -- the extern "C" entry points of libsellcs (declared in include/sellcs.h).
// Every entry point validates its arguments before issuing any HIP call and converts
// every failure into a negative error code; no C++ exception leaves this file.
#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <map>
#include <mutex>
#include <new>
#include <utility>

#include "convert.h"
#include "internal.h"
#include "log.h"

using namespace sellcs;

namespace {

int hip_err(hipError_t e) { return e == hipErrorOutOfMemory ? SELL_ERR_OOM : SELL_ERR_HIP; }

#define HIPCHK(x)                               \
    do {                                        \
        hipError_t e_ = (x);                    \
        if (e_ != hipSuccess) return hip_err(e_); \
    } while (0)

template <class T>
int dev_upload(T **dst, const T *src, size_t n, hipStream_t s) {
    *dst = nullptr;
    if (n == 0) return SELL_OK;
    HIPCHK(lib_malloc(reinterpret_cast<void **>(dst), n * sizeof(T)));
    HIPCHK(hipMemcpyAsync(*dst, src, n * sizeof(T), hipMemcpyHostToDevice, s));
    return SELL_OK;
}

// Frees every device array the matrix holds: also those of a construction that failed half way
// (on_device is only set once an upload is complete).
void free_device(sell_mat *A) {
    if (A->device < 0) return;  // never touched a device (host-only matrix)
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (A->device != cur) (void)hipSetDevice(A->device);
    lib_free(A->d_col);
    lib_free(A->d_val);
    lib_free(A->d_cl);
    lib_free(A->d_cs);
    lib_free(A->d_perm);
    lib_free(A->d_tiles);
    lib_free(A->d_rowslot);
    lib_free(A->d_rowptr);
    lib_free(A->d_tpos);
    A->d_tpos = nullptr;
    lib_free(A->d_stage_np);
    lib_free(A->d_stage_pages);
    lib_free(A->d_stage_own);
    lib_free(A->d_lcol);
    lib_free(A->d_plan_slot);
    lib_free(A->d_plan_miss);
    A->d_stage_np = A->d_stage_pages = A->d_stage_own = nullptr;
    A->d_lcol = nullptr;
    A->d_plan_slot = nullptr;
    A->d_plan_miss = nullptr;
    A->d_col = nullptr;
    A->d_val = nullptr;
    A->d_cl = nullptr;
    A->d_cs = nullptr;
    A->d_perm = nullptr;
    A->d_tiles = nullptr;
    A->d_rowslot = nullptr;
    A->d_rowptr = nullptr;
    if (A->device != cur) (void)hipSetDevice(cur);
}

int upload(sell_mat *A, hipStream_t s) {
    HostSell &h = A->h;
    HIPCHK(hipGetDevice(&A->device));
    int rc;
    if ((rc = dev_upload(&A->d_col, h.col.data(), h.col.size(), s))) return rc;
    if (h.stored > 0) {
        HIPCHK(lib_malloc(&A->d_val, h.val.size()));
        HIPCHK(hipMemcpyAsync(A->d_val, h.val.data(), h.val.size(), hipMemcpyHostToDevice, s));
    }
    if ((rc = dev_upload(&A->d_cl, h.cl.data(), h.cl.size(), s))) return rc;
    if ((rc = dev_upload(&A->d_cs, h.cs.data(), h.cs.size(), s))) return rc;
    if (h.has_perm && (rc = dev_upload(&A->d_perm, h.perm.data(), h.perm.size(), s))) return rc;
    if ((rc = dev_upload(&A->d_tiles, h.tiles.data(), h.tiles.size(), s))) return rc;
    HIPCHK(hipStreamSynchronize(s));
    A->matrix_bytes = int64_t(h.col.size() * 4 + h.val.size() + h.cl.size() * 4 + h.cs.size() * 8 +
                              h.perm.size() * 4 + h.tiles.size() * 4);
    // the device now holds the big arrays; keep only the small metadata on the host
    raw_vector<int32_t>().swap(h.col);
    raw_vector<uint8_t>().swap(h.val);
    A->on_device = true;
    return SELL_OK;
}

// ---- workspace per (device, stream)
std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

}  // namespace

namespace sellcs {

int get_workspace(hipStream_t s, Workspace **ws) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto key = std::make_pair(dev, s);
    auto it = g_ws.find(key);
    if (it != g_ws.end()) {
        *ws = &it->second;
        return SELL_OK;
    }
    Workspace w;
    const size_t np = size_t(kMaxTiles) * 3 * kMaxSliceCols;
    HIPCHK(lib_malloc(&w.partials, np * sizeof(double)));
    if (lib_malloc(&w.scratch, kScratchBytes) != hipSuccess) {
        lib_free(w.partials);
        return SELL_ERR_OOM;
    }
    auto res = g_ws.emplace(key, w);
    *ws = &res.first->second;
    return SELL_OK;
}

void drop_workspace(hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto it = g_ws.find(std::make_pair(dev, s));
    if (it == g_ws.end()) return;
    (void)lib_free(it->second.partials);
    (void)lib_free(it->second.scratch);
    g_ws.erase(it);
}

}  // namespace sellcs

namespace sellcs {

int check_device(const sell_mat *A) {
    if (!A) return SELL_ERR_ARG;
    if (!A->on_device) return SELL_ERR_STATE;
    int cur = -1;
    HIPCHK(hipGetDevice(&cur));
    return cur == A->device ? SELL_OK : SELL_ERR_STATE;
}

int vec_kind(int vdt) {
    return vdt == SELL_F64 ? VK_F64F64 : vdt == SELL_F32 ? VK_F32F32 : VK_BF16F32;
}

int vec_dtype_for(int vdt) { return vdt == SELL_F64 ? SELL_F64 : SELL_F32; }

void bv_strides(const sell_bv *v, int64_t &rs, int64_t &cs) {
    if (v->lay == SELL_ROW_MAJOR) {
        rs = v->ld;
        cs = 1;
    } else {
        rs = 1;
        cs = v->ld;
    }
}

char *elem_ptr(const sell_bv *v, int64_t i, int64_t j) {
    int64_t rs, cs;
    bv_strides(v, rs, cs);
    return static_cast<char *>(v->ptr) + (i * rs + j * cs) * dtype_bytes(v->dt);
}

void base_args(ProdArgs &a, const sell_mat *A) {
    std::memset(&a, 0, sizeof(a));
    a.col = A->d_col;
    a.val = A->d_val;
    a.cl = A->d_cl;
    a.cs = A->d_cs;
    a.perm = A->d_perm;
    a.tiles = A->d_tiles;
    a.ntiles = int32_t(A->h.tiles.size()) - 1;
    if (a.ntiles < 0) a.ntiles = 0;
    a.C = A->h.C;
    a.cshift = -1;
    if ((A->h.C & (A->h.C - 1)) == 0) a.cshift = __builtin_ctz(unsigned(A->h.C));
    a.nrows = A->h.nrows;
    a.ncols_x = A->h.ncols;
    a.alpha = 1.0;
    a.eta = 1.0;
    static const int xcd_map = [] {
        const char *e = std::getenv("SELLCS_XCD_MAP");
        return e ? std::atoi(e) : 1;
    }();
    a.xcd_map = xcd_map;
    a.tile_stride = 0;  // staged launches only: set with the plan
    a.stage = 0;        // set by the product call when the stage arrays and plan fit the launch
    a.st_ntiles = A->stage_ntiles;
    a.st_chunks = A->stage_chunks;
    a.nch = A->h.nch;
    a.st_np = A->d_stage_np;
    a.st_pages = A->d_stage_pages;
    a.st_own = A->d_stage_own;
    a.lcol = A->d_lcol;
    a.vpt_hint = A->vpt_hint;
    a.bpc_hint = A->bpc_hint;
    a.waves_hint = A->waves_hint > 0 ? A->waves_hint : A->h.waves;
    a.batch_hint = A->batch_hint > 0 ? A->batch_hint : A->h.batch;
    a.batch_hint_wide = A->batch_hint > 0 ? A->batch_hint : A->h.batch_wide;
}

// Split b columns into launches: slices of width `hint` when it divides b (a width chosen for
// the matrix, e.g. by the autotuner), else fixed widths when possible, else up to 64 per launch.
std::vector<std::pair<int, int>> slices(int b, int hint = 0) {
    std::vector<std::pair<int, int>> out;
    if (hint > 0 && hint < b && b % hint == 0) {
        for (int j = 0; j < b; j += hint) out.emplace_back(j, hint);
        return out;
    }
    auto fixed = [](int w) { return w == 1 || w == 2 || w == 4 || w == 8 || w == 16 || w == 32; };
    if (fixed(b) || b <= kMaxSliceCols) {
        out.emplace_back(0, b);
        return out;
    }
    int j = 0;
    while (b - j > kMaxSliceCols) {
        out.emplace_back(j, 32);
        j += 32;
    }
    out.emplace_back(j, b - j);
    return out;
}

int validate_bv(const sell_bv *v) {
    if (!v || (!v->ptr && v->nrows * int64_t(v->ncols) > 0)) return SELL_ERR_ARG;
    return SELL_OK;
}


// y = alpha (A x - gamma x) + beta y, dots, chain; no argument checks (callers check).
int aug_impl(const sell_mat *A, const sell_bv *X, sell_bv *Y, sell_bv *Z, const sell_spmv_opts &o,
             bool aug, hipStream_t s, double *partials_out, int32_t *nblocks_out, const Workspace *ws_in) {
    if (nblocks_out) *nblocks_out = 0;
    const int b = X->ncols;
    const bool dots = aug && (o.flags & SELL_SPMV_DOTS);
    // x through LDS: stage tiles of one pass of the kernel (kBlock * columns per lane / b rows)
    // for the fixed widths whose rows are at least 16 bytes, one workgroup per compute unit and
    // a precomputed slot plan. A caller that brings its own workspace may not allocate: it runs
    // staged only when the arrays and the plan already fit the launch.
    bool staged = false;
    int32_t st_nblk = 0, st_stride = 0;
    const int xbytes_row = b * (A->h.vdt == SELL_F64 ? 8 : 4);
    if (A->stage_hint && A->h.nrows > 0 && (b == 2 || b == 4 || b == 8 || b == 16 || b == 32) && xbytes_row >= 16 &&
        (partials_out || slices(b, A->slice_hint).size() == 1)) {
        const int vpt = choose_vpt(vec_kind(A->h.vdt), b, A->vpt_hint);
        const int32_t chunks = std::max<int32_t>(1, int32_t(kBlock * vpt / b) / A->h.C);
        const int32_t ns = std::min<int32_t>(kStageMaxPages, kStageBytes / (kStagePage * xbytes_row));
        int ncu = 0, dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
            ncu = 256;
        int rc = SELL_OK;
        if (!A->d_lcol || A->stage_chunks != chunks) rc = ws_in ? SELL_ERR_STATE : ensure_stage(A, chunks, s);
        if (rc == SELL_OK) {
            const int64_t units = A->stage_ntiles;
            st_nblk = int32_t(std::min<int64_t>(ncu, units));
            st_stride = A->tile_stride_hint;
            if (st_stride > 0 && (units % st_stride || st_nblk % st_stride)) st_stride = 0;
            if (!(A->d_plan_slot && A->plan_nblk == st_nblk && A->plan_stride == st_stride && A->plan_ns == ns))
                rc = ws_in ? SELL_ERR_STATE : ensure_stage_plan(A, st_nblk, st_stride, ns, s);
        }
        if (rc == SELL_OK)
            staged = true;
        else if (!ws_in)
            return rc;
    }
    const Workspace *ws = ws_in;
    if (!ws) {
        Workspace *w = nullptr;
        int rc = get_workspace(s, &w);
        if (rc) return rc;
        ws = w;
    }
    if (A->h.nrows == 0 || A->h.tiles.size() < 2) {
        // empty matrix: y is empty; dots of empty columns are zero
        if (dots) {
            if (partials_out) return SELL_OK;  // no tiles: nothing to sum
            const uint32_t g[3] = {SELL_SPMV_DOT_YY, SELL_SPMV_DOT_XY, SELL_SPMV_DOT_XX};
            for (int q = 0; q < 3; ++q)
                if (o.flags & g[q]) {
                    int rc = launch_fill(o.dot + q * b, SELL_F64, 1, b, b, 1, 0.0, s);
                    if (rc) return rc;
                }
        }
        return SELL_OK;
    }
    // the solvers (partials_out) need one slice: they ignore the matrix's slice width
    auto sl_list = slices(b, partials_out ? 0 : A->slice_hint);
    if (partials_out && sl_list.size() != 1) return SELL_ERR_UNSUPPORTED;
    for (auto sl : sl_list) {
        ProdArgs a;
        base_args(a, A);
        a.nb = sl.second;
        bv_strides(X, a.xrs, a.xcs);
        bv_strides(Y, a.yrs, a.ycs);
        a.X = elem_ptr(X, 0, sl.first);
        a.Y = elem_ptr(Y, 0, sl.first);
        a.scratch = ws->scratch;
        a.stage = staged ? 1 : 0;
        if (staged) {
            a.tile_stride = st_stride;
            a.st_nblocks = st_nblk;
            a.st_slot = A->d_plan_slot;
            a.st_miss = A->d_plan_miss;
        }
        if (aug && (o.flags & SELL_SPMV_CHAIN)) {
            bv_strides(Z, a.zrs, a.zcs);
            a.Z = elem_ptr(Z, 0, sl.first);
        }
        if (aug) {
            a.flags = o.flags;
            a.alpha = o.alpha;
            a.beta = o.beta;
            a.delta = o.delta;
            a.eta = o.eta;
            a.gamma_s = o.gamma;
            if (o.flags & SELL_SPMV_VSHIFT) {
                a.has_gamma_v = 1;
                for (int j = 0; j < sl.second; ++j) a.gamma_v[j] = o.gamma_v[sl.first + j];
            }
            if (dots) a.partials = partials_out ? partials_out : ws->partials;
        }
        int rc = launch_product(a, vec_kind(A->h.vdt), aug, s);
        if (rc) return rc;
        if (nblocks_out) *nblocks_out = a.nblocks;
        if (dots && !partials_out) {
            rc = launch_dot_finish(ws->partials, a.nblocks, a.nb, o.flags, o.dot + sl.first, b, 1, 0, s);
            if (rc) return rc;
        }
    }
    return SELL_OK;
}

}  // namespace sellcs

namespace {

int check_product_operands(const sell_mat *A, const sell_bv *X, const sell_bv *Y) {
    int rc = check_device(A);
    if (rc) return rc;
    if ((rc = validate_bv(X)) || (rc = validate_bv(Y))) return rc;
    const int vdt = vec_dtype_for(A->h.vdt);
    if (X->dt != vdt || Y->dt != vdt) return SELL_ERR_DTYPE;
    if (X->ncols != Y->ncols || X->ncols < 1) return SELL_ERR_SHAPE;
    return SELL_OK;
}

// SELLCS_LOG >= 2: what a build made
void log_built(const sell_mat *M, const char *where) {
    if (log_level() < 2) return;
    const HostSell &h = M->h;
    static const char *const kType[] = {"f64", "f32", "bf16"};
    log_info("built SELL-%d-%lld %s: %lld x %lld, %lld nonzeros, %lld stored (%.4f per nonzero), %lld chunks, "
             "%d tiles, %s values, index batch %d (%d for 32-byte lanes), grid of %d wave(s)",
             int(h.C), (long long)h.sigma, where, (long long)h.nrows, (long long)h.ncols, (long long)h.nnz,
             (long long)h.stored, h.nnz > 0 ? double(h.stored) / double(h.nnz) : 1.0, (long long)h.nch,
             int(M->ntiles), h.vdt >= 0 && h.vdt <= 2 ? kType[h.vdt] : "?", int(h.batch), int(h.batch_wide),
             int(h.waves));
}

int build_common(sell_mat **A, int64_t nrows, int64_t ncols, const int64_t *rowptr, const int32_t *col,
                 const double *val, int32_t C, int64_t sigma, sell_dtype vdt, bool device, hipStream_t s) {
    if (!A) return SELL_ERR_ARG;
    *A = nullptr;
    sell_mat *M = new (std::nothrow) sell_mat();
    if (!M) return SELL_ERR_OOM;
    int rc;
    try {
        rc = build_host_sell(M->h, nrows, ncols, rowptr, col, val, C, sigma, int(vdt));
    } catch (const std::bad_alloc &) {
        rc = SELL_ERR_OOM;
    } catch (...) {
        rc = SELL_ERR_ARG;
    }
    if (rc) {
        delete M;
        return rc;
    }
    M->ntiles = int32_t(M->h.tiles.size()) - 1;
    if (device) {
        rc = upload(M, s);
        if (rc) {
            free_device(M);
            delete M;
            return rc;
        }
    }
    log_built(M, device ? "from host CSR" : "in host memory only");
    *A = M;
    return SELL_OK;
}

}  // namespace

extern "C" {

const char *sell_strerror(int code) {
    switch (code) {
        case SELL_OK: return "success";
        case SELL_ERR_ARG: return "invalid argument";
        case SELL_ERR_SHAPE: return "operand shapes do not match";
        case SELL_ERR_DTYPE: return "unsupported element-type combination";
        case SELL_ERR_UNSUPPORTED: return "unsupported request";
        case SELL_ERR_OOM: return "out of memory";
        case SELL_ERR_HIP: return "HIP runtime error";
        case SELL_ERR_STATE: return "object not usable here (host-only or other device)";
        default: return "unknown error";
    }
}

int sell_version(void) { return 10000 * 1 + 100 * 0 + 0; }

int sell_build(sell_mat **A, int64_t nrows, int64_t ncols, const int64_t *rowptr, const int32_t *col,
               const double *val, int32_t C, int64_t sigma, sell_dtype vdt, void *stream) {
    return build_common(A, nrows, ncols, rowptr, col, val, C, sigma, vdt, true,
                        static_cast<hipStream_t>(stream));
}

int sell_build_device(sell_mat **A, int64_t nrows, int64_t ncols, const int64_t *rowptr, const int32_t *col,
                      const double *val, int32_t C, int64_t sigma, sell_dtype vdt, void *stream) {
    if (!A) return SELL_ERR_ARG;
    *A = nullptr;
    sell_mat *M = new (std::nothrow) sell_mat();
    if (!M) return SELL_ERR_OOM;
    int rc;
    try {
        rc = build_device_sell(M, nrows, ncols, rowptr, col, val, C, sigma, int(vdt), static_cast<hipStream_t>(stream));
    } catch (const std::bad_alloc &) {
        rc = SELL_ERR_OOM;
    }
    if (rc) {
        M->on_device = true;  // release whatever device arrays the build made
        free_device(M);
        delete M;
        return rc;
    }
    log_built(M, "on the device");
    *A = M;
    return SELL_OK;
}

int sell_build_host(sell_mat **A, int64_t nrows, int64_t ncols, const int64_t *rowptr,
                    const int32_t *col, const double *val, int32_t C, int64_t sigma, sell_dtype vdt) {
    return build_common(A, nrows, ncols, rowptr, col, val, C, sigma, vdt, false, nullptr);
}

int sell_destroy(sell_mat *A) {
    if (!A) return SELL_OK;
    if (A->transpose) sell_destroy(A->transpose);
    free_device(A);
    delete A;
    return SELL_OK;
}

int sell_info(const sell_mat *A, sell_info_t *o) {
    if (!A || !o) return SELL_ERR_ARG;
    o->nrows = A->h.nrows;
    o->ncols = A->h.ncols;
    o->nnz = A->h.nnz;
    o->stored = A->h.stored;
    o->nchunks = A->h.nch;
    o->sigma = A->h.sigma;
    o->C = A->h.C;
    o->vdtype = A->h.vdt;
    o->on_device = A->on_device ? 1 : 0;
    o->device = A->on_device ? A->device : -1;
    o->ntiles = A->ntiles;
    o->has_perm = A->h.has_perm ? 1 : 0;
    o->matrix_bytes = A->on_device ? A->matrix_bytes
                                   : int64_t(A->h.col.size() * 4 + A->h.val.size() + A->h.cl.size() * 4 +
                                             A->h.cs.size() * 8 + A->h.perm.size() * 4);
    o->batch = A->batch_hint > 0 ? A->batch_hint : A->h.batch;
    o->batch_wide = A->batch_hint > 0 ? A->batch_hint : A->h.batch_wide;
    return SELL_OK;
}

int sell_export_sell(const sell_mat *A, int32_t *perm, int32_t *cl, int64_t *cs, int32_t *col, double *val) {
    if (!A) return SELL_ERR_ARG;
    const HostSell &h = A->h;
    try {
        if (perm) {
            if (h.has_perm)
                std::copy(h.perm.begin(), h.perm.end(), perm);
            else
                for (int64_t s = 0; s < h.nch * h.C; ++s) perm[s] = s < h.nrows ? int32_t(s) : -1;
        }
        if (cl) std::copy(h.cl.begin(), h.cl.end(), cl);
        if (cs) std::copy(h.cs.begin(), h.cs.end(), cs);
        if (!col && !val) return SELL_OK;
        std::vector<int32_t> dcol;
        std::vector<uint8_t> dval;
        const int32_t *pc = h.col.data();
        const uint8_t *pv = h.val.data();
        if (A->on_device) {
            dcol.resize(size_t(h.stored));
            dval.resize(size_t(h.stored) * dtype_bytes(h.vdt));
            if (h.stored > 0) {
                HIPCHK(hipMemcpy(dcol.data(), A->d_col, dcol.size() * 4, hipMemcpyDeviceToHost));
                HIPCHK(hipMemcpy(dval.data(), A->d_val, dval.size(), hipMemcpyDeviceToHost));
            }
            pc = dcol.data();
            pv = dval.data();
        }
        if (col) std::copy(pc, pc + h.stored, col);
        if (val) {
            for (int64_t e = 0; e < h.stored; ++e) {
                if (h.vdt == SELL_F64)
                    std::memcpy(&val[e], pv + e * 8, 8);
                else if (h.vdt == SELL_F32) {
                    float f;
                    std::memcpy(&f, pv + e * 4, 4);
                    val[e] = f;
                } else {
                    uint16_t u;
                    std::memcpy(&u, pv + e * 2, 2);
                    val[e] = f32_from_bf16(u);
                }
            }
        }
    } catch (const std::bad_alloc &) {
        return SELL_ERR_OOM;
    }
    return SELL_OK;
}

int sell_export_csr(const sell_mat *A, int64_t *rowptr, int32_t *col, double *val) {
    if (!A || !rowptr) return SELL_ERR_ARG;
    const HostSell &h = A->h;
    if (h.nnz > 0 && (!col || !val)) return SELL_ERR_ARG;
    try {
        std::vector<int32_t> scol(static_cast<size_t>(h.stored));
        std::vector<double> sval(static_cast<size_t>(h.stored));
        int rc = sell_export_sell(A, nullptr, nullptr, nullptr, scol.data(), sval.data());
        if (rc) return rc;
        std::copy(h.rowptr.begin(), h.rowptr.end(), rowptr);
        for (int64_t slot = 0; slot < h.nch * h.C; ++slot) {
            const int64_t row = h.has_perm ? h.perm[slot] : (slot < h.nrows ? slot : -1);
            if (row < 0) continue;
            const int64_t c = slot / h.C, r = slot % h.C;
            const int64_t p0 = h.rowptr[row], len = h.rowptr[row + 1] - p0;
            for (int64_t k = 0; k < len; ++k) {
                col[p0 + k] = scol[h.cs[c] + k * h.C + r];
                val[p0 + k] = sval[h.cs[c] + k * h.C + r];
            }
        }
    } catch (const std::bad_alloc &) {
        return SELL_ERR_OOM;
    }
    return SELL_OK;
}

}  // extern "C"

namespace sellcs {
int ensure_update_maps(sell_mat *A, hipStream_t s) {
    if (A->d_rowptr) return SELL_OK;
    const HostSell &h = A->h;
    std::vector<int32_t> rowslot(static_cast<size_t>(h.nrows));
    for (int64_t slot = 0; slot < h.nch * h.C; ++slot) {
        const int64_t row = h.has_perm ? h.perm[slot] : (slot < h.nrows ? slot : -1);
        if (row >= 0) rowslot[row] = int32_t(slot);
    }
    // both maps are built before either is published: d_rowptr marks them as present, so a
    // failure half way must not leave it set
    int64_t *rp = nullptr;
    int32_t *rs = nullptr;
    int rc = dev_upload(&rp, h.rowptr.data(), h.rowptr.size(), s);
    if (!rc) rc = dev_upload(&rs, rowslot.data(), rowslot.size(), s);
    if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = SELL_ERR_HIP;
    if (rc) {
        (void)hipStreamSynchronize(s);
        (void)lib_free(rp);
        (void)lib_free(rs);
        return rc;
    }
    A->d_rowptr = rp;
    A->d_rowslot = rs;
    return SELL_OK;
}
}  // namespace sellcs

extern "C" {

int sell_update_values_device(sell_mat *A, const double *val, void *stream) {
    int rc = check_device(A);
    if (rc) return rc;
    if (!val && A->h.nnz > 0) return SELL_ERR_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    try {
        if ((rc = ensure_update_maps(A, s))) return rc;
    } catch (const std::bad_alloc &) {
        return SELL_ERR_OOM;
    }
    if ((rc = launch_update_values(A, val, s))) return rc;
    // keep the SELL copy of A^T in step: every value goes straight to its slot there
    if (A->transpose && A->h.nnz > 0)
        rc = launch_scatter_values(val, A->d_tpos, A->h.nnz, A->transpose->h.vdt, A->transpose->d_val, s);
    return rc;
}

int sell_update_values(sell_mat *A, const double *val, void *stream) {
    if (!A) return SELL_ERR_ARG;
    if (!val && A->h.nnz > 0) return SELL_ERR_ARG;
    if (!A->on_device) {
        // host-only matrix: scatter into the host arrays
        HostSell &h = A->h;
        std::vector<double> sval(size_t(h.stored), 0.0);
        for (int64_t slot = 0; slot < h.nch * h.C; ++slot) {
            const int64_t row = h.has_perm ? h.perm[slot] : (slot < h.nrows ? slot : -1);
            if (row < 0) continue;
            const int64_t c = slot / h.C, r = slot % h.C;
            const int64_t p0 = h.rowptr[row], len = h.rowptr[row + 1] - p0;
            for (int64_t k = 0; k < len; ++k) sval[h.cs[c] + k * h.C + r] = val[p0 + k];
        }
        convert_values(sval.data(), h.stored, h.vdt, h.val.data());
        return SELL_OK;
    }
    int rc = check_device(A);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (A->h.nnz == 0) return SELL_OK;
    double *d = nullptr;
    HIPCHK(lib_malloc(&d, size_t(A->h.nnz) * sizeof(double)));
    hipError_t e = hipMemcpyAsync(d, val, size_t(A->h.nnz) * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) rc = sell_update_values_device(A, d, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    lib_free(d);
    if (e != hipSuccess) return hip_err(e);
    return rc;
}

// ---------------------------------------------------------------- block vectors

int sell_bv_create(sell_bv **X, int64_t nrows, int32_t ncols, sell_dtype dt, sell_layout lay, void *data,
                   int64_t ld) {
    if (!X) return SELL_ERR_ARG;
    *X = nullptr;
    if (nrows < 0 || ncols < 1) return SELL_ERR_ARG;
    if (dt != SELL_F64 && dt != SELL_F32 && dt != SELL_BF16) return SELL_ERR_DTYPE;
    if (lay != SELL_ROW_MAJOR && lay != SELL_COL_MAJOR) return SELL_ERR_ARG;
    sell_bv *v = new (std::nothrow) sell_bv();
    if (!v) return SELL_ERR_OOM;
    v->nrows = nrows;
    v->ncols = ncols;
    v->dt = dt;
    v->lay = lay;
    if (hipGetDevice(&v->device) != hipSuccess) {
        delete v;
        return SELL_ERR_HIP;
    }
    if (data) {
        const int64_t minld = lay == SELL_ROW_MAJOR ? ncols : nrows;
        if (ld < minld || ld < 1) {
            delete v;
            return SELL_ERR_ARG;
        }
        v->ptr = data;
        v->ld = ld;
        v->owned = false;
    } else {
        v->ld = lay == SELL_ROW_MAJOR ? ncols : std::max<int64_t>(nrows, 1);
        const size_t bytes = size_t(nrows) * size_t(ncols) * dtype_bytes(dt);
        if (bytes > 0) {
            hipError_t e = lib_malloc(&v->ptr, bytes);
            if (e == hipSuccess) e = hipMemset(v->ptr, 0, bytes);
            if (e != hipSuccess) {
                lib_free(v->ptr);
                delete v;
                return hip_err(e);
            }
        }
        v->owned = true;
    }
    *X = v;
    return SELL_OK;
}

int sell_bv_destroy(sell_bv *X) {
    if (!X) return SELL_OK;
    if (X->owned && X->ptr) lib_free(X->ptr);
    delete X;
    return SELL_OK;
}

int sell_bv_data(const sell_bv *X, void **data, int64_t *ld, int64_t *nrows, int32_t *ncols, int32_t *dtype,
                 int32_t *layout) {
    if (!X) return SELL_ERR_ARG;
    if (data) *data = X->ptr;
    if (ld) *ld = X->ld;
    if (nrows) *nrows = X->nrows;
    if (ncols) *ncols = X->ncols;
    if (dtype) *dtype = X->dt;
    if (layout) *layout = X->lay;
    return SELL_OK;
}

int sell_bv_copy(sell_bv *dst, const sell_bv *src, void *stream) {
    int rc;
    if ((rc = validate_bv(dst)) || (rc = validate_bv(src))) return rc;
    if (dst->nrows != src->nrows || dst->ncols != src->ncols) return SELL_ERR_SHAPE;
    if (dst == src) return SELL_OK;
    return launch_copy(dst, src, static_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------------- products

int sell_spmmv(const sell_mat *A, const sell_bv *X, sell_bv *Y, void *stream) {
    int rc = check_product_operands(A, X, Y);
    if (rc) return rc;
    if (X->nrows != A->h.ncols || Y->nrows != A->h.nrows) return SELL_ERR_SHAPE;
    if (X->ptr == Y->ptr && A->h.nrows > 0) return SELL_ERR_ARG;
    sell_spmv_opts o = SELL_SPMV_OPTS_INIT;
    return aug_impl(A, X, Y, nullptr, o, false, static_cast<hipStream_t>(stream));
}

int sell_spmmv_aug(const sell_mat *A, const sell_bv *X, sell_bv *Y, sell_bv *Z, const sell_spmv_opts *opts,
                   void *stream) {
    sell_spmv_opts o;
    int rc = check_aug_call(A, X, Y, Z, opts, &o);
    if (rc) return rc;
    const bool plain = (o.flags == 0);
    return aug_impl(A, X, Y, Z, o, !plain, static_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace sellcs {
int check_aug_call(const sell_mat *A, const sell_bv *X, sell_bv *Y, sell_bv *Z, const sell_spmv_opts *opts,
                   sell_spmv_opts *out) {
    int rc = check_product_operands(A, X, Y);
    if (rc) return rc;
    sell_spmv_opts o = SELL_SPMV_OPTS_INIT;
    if (opts) o = *opts;
    const uint32_t known = 0xFFu;
    if (o.flags & ~known) return SELL_ERR_ARG;
    if (X->nrows != A->h.ncols || Y->nrows != A->h.nrows) return SELL_ERR_SHAPE;
    const uint32_t sq = SELL_SPMV_SHIFT | SELL_SPMV_VSHIFT | SELL_SPMV_DOT_XY | SELL_SPMV_DOT_XX;
    if ((o.flags & sq) && A->h.nrows != A->h.ncols) return SELL_ERR_SHAPE;
    if ((o.flags & SELL_SPMV_VSHIFT) && !o.gamma_v) return SELL_ERR_ARG;
    if ((o.flags & SELL_SPMV_DOTS) && !o.dot) return SELL_ERR_ARG;
    if (X->ptr == Y->ptr && A->h.nrows > 0) return SELL_ERR_ARG;
    if (o.flags & SELL_SPMV_CHAIN) {
        if ((rc = validate_bv(Z))) return rc;
        if (Z->dt != Y->dt) return SELL_ERR_DTYPE;
        if (Z->nrows != Y->nrows || Z->ncols != Y->ncols) return SELL_ERR_SHAPE;
        if (Z->ptr == Y->ptr && A->h.nrows > 0) return SELL_ERR_ARG;
    }
    *out = o;
    return SELL_OK;
}

int ensure_transpose(const sell_mat *A, hipStream_t s) {
    if (A->transpose) return SELL_OK;
    const HostSell &h = A->h;
    std::vector<int64_t> rp(size_t(h.nrows) + 1);
    std::vector<int32_t> col(static_cast<size_t>(h.nnz));
    std::vector<double> val(static_cast<size_t>(h.nnz));
    // the export reads the device values with blocking copies on the null stream, which do not
    // wait for work on a non-blocking stream: a value update still queued on s must land first
    if (A->on_device) {
        const hipError_t se = hipStreamSynchronize(s);
        if (se != hipSuccess) return hip_err(se);
    }
    int rc = sell_export_csr(A, rp.data(), col.data(), val.data());
    if (rc) return rc;
    // CSR of A^T by a counting sort over columns (rows stay ascending inside each column);
    // tpos[p] records where entry p of A lands, for later value updates
    std::vector<int64_t> trp(size_t(h.ncols) + 1, 0);
    for (int64_t p = 0; p < h.nnz; ++p) trp[size_t(col[p]) + 1]++;
    for (int64_t c = 0; c < h.ncols; ++c) trp[c + 1] += trp[c];
    std::vector<int64_t> fill(trp.begin(), trp.end() - 1);
    std::vector<int32_t> tcol(static_cast<size_t>(h.nnz));
    std::vector<double> tval(static_cast<size_t>(h.nnz));
    std::vector<int64_t> tpos(static_cast<size_t>(h.nnz));
    for (int64_t i = 0; i < h.nrows; ++i)
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            const int64_t at = fill[col[p]]++;
            tcol[at] = int32_t(i);
            tval[at] = val[p];
            tpos[p] = at;
        }
    sell_mat *T = nullptr;
    rc = build_common(&T, h.ncols, h.nrows, trp.data(), tcol.data(), tval.data(), h.C, h.sigma,
                      sell_dtype(h.vdt), true, s);
    if (rc) return rc;
    // turn the A^T CSR positions into A^T SELL positions, so that a value update of A
    // refreshes the copy with one scatter
    {
        const HostSell &th = T->h;
        std::vector<int64_t> slot_of(static_cast<size_t>(th.nrows));
        for (int64_t slot = 0; slot < th.nch * th.C; ++slot) {
            const int64_t row = th.has_perm ? th.perm[slot] : (slot < th.nrows ? slot : -1);
            if (row >= 0) slot_of[row] = slot;
        }
        std::vector<int64_t> sell_of_q(static_cast<size_t>(h.nnz));
        for (int64_t t = 0; t < th.nrows; ++t) {
            const int64_t c = slot_of[t] / th.C, r = slot_of[t] % th.C;
            for (int64_t q = th.rowptr[t]; q < th.rowptr[t + 1]; ++q)
                sell_of_q[q] = th.cs[c] + (q - th.rowptr[t]) * th.C + r;
        }
        for (int64_t p = 0; p < h.nnz; ++p) tpos[p] = sell_of_q[tpos[p]];
    }
    sell_mat *M = const_cast<sell_mat *>(A);
    rc = dev_upload(&M->d_tpos, tpos.data(), tpos.size(), s);
    if (rc == SELL_OK && hipStreamSynchronize(s) != hipSuccess) rc = SELL_ERR_HIP;
    if (rc) {
        sell_destroy(T);
        lib_free(M->d_tpos);
        M->d_tpos = nullptr;
        return rc;
    }
    M->transpose = T;
    return SELL_OK;
}

}  // namespace sellcs

extern "C" {

int sell_spmmv_T(const sell_mat *A, const sell_bv *X, sell_bv *Y, int deterministic, void *stream) {
    int rc = check_product_operands(A, X, Y);
    if (rc) return rc;
    if (X->nrows != A->h.nrows || Y->nrows != A->h.ncols) return SELL_ERR_SHAPE;
    if (X->ptr == Y->ptr && A->h.nrows > 0) return SELL_ERR_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (deterministic) {
        try {
            if ((rc = ensure_transpose(A, s))) return rc;
        } catch (const std::bad_alloc &) {
            return SELL_ERR_OOM;
        }
        sell_spmv_opts o = SELL_SPMV_OPTS_INIT;
        return aug_impl(A->transpose, X, Y, nullptr, o, false, s);
    }
    log_warn_once(kWarnAtomicTranspose,
                  "transposed product by atomic scatter (deterministic = 0): it is much slower than the "
                  "deterministic transpose, which builds a SELL copy of the transpose once per matrix");
    int64_t yrs, ycs;
    bv_strides(Y, yrs, ycs);
    if ((rc = launch_fill(Y->ptr, Y->dt, Y->nrows, Y->ncols, yrs, ycs, 0.0, s))) return rc;
    if (A->h.nrows == 0 || A->ntiles == 0) return SELL_OK;
    for (auto sl : slices(X->ncols)) {
        ProdArgs a;
        base_args(a, A);
        a.nb = sl.second;
        bv_strides(X, a.xrs, a.xcs);
        bv_strides(Y, a.yrs, a.ycs);
        a.X = elem_ptr(X, 0, sl.first);
        a.Y = elem_ptr(Y, 0, sl.first);
        if ((rc = launch_transpose_atomic(a, vec_kind(A->h.vdt), s))) return rc;
    }
    return SELL_OK;
}

// ---------------------------------------------------------------- KPM driver

int sell_kpm(const sell_mat *A, sell_bv *V, sell_bv *W, int64_t M, double scale, double c, double *mu,
             int *last_in_w, float *step_ms, void *stream) {
    int rc = check_product_operands(A, V, W);
    if (rc) return rc;
    if (A->h.vdt != SELL_F64) return SELL_ERR_DTYPE;
    if (A->h.nrows != A->h.ncols || V->nrows != A->h.nrows || W->nrows != A->h.nrows) return SELL_ERR_SHAPE;
    if (M < 1 || !mu || !(scale != 0.0) || !std::isfinite(scale) || !std::isfinite(c)) return SELL_ERR_ARG;
    if (V->ptr == W->ptr && A->h.nrows > 0) return SELL_ERR_ARG;
    const int b = V->ncols;
    if (b > kMaxSliceCols) return SELL_ERR_UNSUPPORTED;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // timing events come from a per-thread, per-device pool that lives as long as the process,
    // so a timed call creates none (creating a few hundred events costs about a millisecond of
    // host time, during which the device would wait)
    std::vector<hipEvent_t> ev;
    if (step_ms) {
        static thread_local std::map<int, std::vector<hipEvent_t>> pools;
        int dev = 0;
        HIPCHK(hipGetDevice(&dev));
        std::vector<hipEvent_t> &pool = pools[dev];
        while (pool.size() < size_t(M) + 1) {
            hipEvent_t e = nullptr;
            // timing only (read after a stream synchronisation): no system-scope fence with its
            // cache writeback and invalidation at every record (a 200-product step at b = 8 on the
            // 128^3 Anderson matrix: 27.68 ms with fenced events, 27.00 fence-free, 26.49 without)
            HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
            pool.push_back(e);
        }
        ev.assign(pool.begin(), pool.begin() + (size_t(M) + 1));
    }
    // per-step tile partials of the dots, summed once after the recurrence
    const int32_t nt = A->ntiles;
    const size_t per_step = size_t(3) * b * size_t(nt > 0 ? nt : 1);
    double *dots = nullptr, *parts = nullptr;
    hipError_t e = lib_malloc_async(reinterpret_cast<void **>(&dots), size_t(M) * 3 * b * sizeof(double), s);
    if (e == hipSuccess) e = lib_malloc_async(reinterpret_cast<void **>(&parts), size_t(M) * per_step * sizeof(double), s);
    if (e != hipSuccess) rc = hip_err(e);
    sell_spmv_opts o = SELL_SPMV_OPTS_INIT;
    // v1 = (A v0 - c v0) / s, with <v1,v1>, <v0,v1>, <v0,v0>
    o.flags = SELL_SPMV_SCALE | SELL_SPMV_SHIFT | SELL_SPMV_DOTS;
    o.alpha = 1.0 / scale;
    o.gamma = c;
    if (rc == SELL_OK && step_ms) (void)hipEventRecord(ev[0], s);
    int32_t nblk = 0, nblk1 = 0;
    if (rc == SELL_OK) rc = aug_impl(A, V, W, nullptr, o, true, s, parts, &nblk);
    if (rc == SELL_OK && step_ms) (void)hipEventRecord(ev[1], s);
    sell_bv *x = W, *y = V;  // x = v_m, y = v_{m-1} -> v_{m+1}
    o.flags = SELL_SPMV_SCALE | SELL_SPMV_SHIFT | SELL_SPMV_AXPBY | SELL_SPMV_DOT_YY | SELL_SPMV_DOT_XY;
    o.alpha = 2.0 / scale;
    o.beta = -1.0;
    for (int64_t m = 1; m < M && rc == SELL_OK; ++m) {
        rc = aug_impl(A, x, y, nullptr, o, true, s, parts + size_t(m) * per_step, &nblk1);
        if (rc == SELL_OK && step_ms) (void)hipEventRecord(ev[size_t(m) + 1], s);
        std::swap(x, y);
    }
    // the first step and the later ones (the same flags each, hence the same launch shape) left
    // nblk and nblk1 partials per quantity, 3 b quantities, at the start of each step's region
    if (rc == SELL_OK && A->h.nrows > 0 && nblk > 0) {
        rc = launch_dot_finish_strided(parts, nblk, b, SELL_SPMV_DOTS, dots, b, 1, 3 * b, per_step, s);
        if (rc == SELL_OK && M > 1)
            rc = launch_dot_finish_strided(parts + per_step, nblk1, b, SELL_SPMV_DOTS, dots + 3 * b, b, M - 1, 3 * b,
                                           per_step, s);
    } else if (rc == SELL_OK)
        rc = launch_fill(dots, SELL_F64, M, 3 * b, 3 * b, 1, 0.0, s);
    if (rc == SELL_OK) rc = launch_kpm_moments(dots, M, b, mu, s);
    if (parts) {
        e = lib_free_async(parts, s);
        if (rc == SELL_OK && e != hipSuccess) rc = hip_err(e);
    }
    if (dots) {
        e = lib_free_async(dots, s);
        if (rc == SELL_OK && e != hipSuccess) rc = hip_err(e);
    }
    if (step_ms) {
        if (rc == SELL_OK) {
            e = hipStreamSynchronize(s);
            if (e != hipSuccess) rc = hip_err(e);
        }
        for (int64_t m = 0; m < M && rc == SELL_OK; ++m) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, ev[size_t(m)], ev[size_t(m) + 1]);
            if (e != hipSuccess) rc = hip_err(e);
            step_ms[m] = ms;
        }
    }
    if (last_in_w) *last_in_w = (x == W) ? 1 : 0;
    return rc;
}

// ---------------------------------------------------------------- probes

int sell_probe_bandwidth(int kind, void *dst, const void *src, int64_t bytes, void *stream) {
    if (kind < 0 || kind > 4 || bytes <= 0 || bytes % 16 != 0 || !dst) return SELL_ERR_ARG;
    if (kind != 2 && kind != 4 && !src) return SELL_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) & 15u) return SELL_ERR_ARG;
    return launch_probe(kind, dst, src, bytes, static_cast<hipStream_t>(stream));
}

int sell_probe_stream(int reads, int writes, int unroll, int nontemporal, int grid, void *dst, const void *src,
                      int64_t bytes, void *stream) {
    if (reads < 0 || reads > 4 || writes < 0 || writes > 1 || reads + writes < 1) return SELL_ERR_ARG;
    if (unroll != 1 && unroll != 2 && unroll != 4 && unroll != 8) return SELL_ERR_ARG;
    if (grid < 1 || grid > (1 << 20) || bytes <= 0 || bytes % 16 != 0 || !dst) return SELL_ERR_ARG;
    if (reads > 0 && !src) return SELL_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) & 15u) return SELL_ERR_ARG;
    return launch_probe_stream(reads, writes, unroll, nontemporal, grid, dst, src, bytes,
                               static_cast<hipStream_t>(stream));
}

}  // extern "C"
