// cheb.cpp -- derivatives with respect to the stored matrix values.
//
//  * sell_grad_values: dL/dval for Y = A X given G = dL/dY (pattern-restricted outer product).
//  * sell_cheb_filter: Z = sum_m coef_m T_m(A~) X, the chained axpby of the augmented product
//    accumulating z = z + coef_m+1 v_m+1 in the step that forms v_m+1.
//  * sell_cheb_forward / sell_cheb_backward: Y = T_N(A~) X with A~ = (A - c I) / s by the
//    three-term Chebyshev recurrence (each step one augmented product), and its adjoint.
//    The forward pass keeps the pair (v_kK, v_kK+1) every K steps; the backward pass walks
//    the segments from the last to the first, recomputes each segment's vectors from its
//    checkpoint and runs the adjoint recurrence
//        w_m += 2 A~^T w_m+1,   w_m-1 -= w_m+1,   dval += (2/s) outer(w_m+1, v_m)
//    (A~^T w via the forward kernel on the SELL copy of A^T, fused with the scaling, the shift
//    and the accumulation in one augmented product), ending with the first step v_1 = A~ v_0.
#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

#include "internal.h"

using namespace sellcs;

namespace {

#define HIPCHK(x)                                                                             \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess) return e_ == hipErrorOutOfMemory ? SELL_ERR_OOM : SELL_ERR_HIP; \
    } while (0)

int vec_dt_of(const sell_mat *A) { return A->h.vdt == SELL_F64 ? SELL_F64 : SELL_F32; }

int check_block(const sell_mat *A, const sell_bv *v, int64_t nrows, int b) {
    if (!v) return SELL_ERR_ARG;
    if (v->dt != vec_dt_of(A)) return SELL_ERR_DTYPE;
    if (v->nrows != nrows || v->ncols != b) return SELL_ERR_SHAPE;
    if (v->lay != SELL_ROW_MAJOR || v->ld != v->ncols) return SELL_ERR_UNSUPPORTED;
    if (!v->ptr && nrows * b > 0) return SELL_ERR_ARG;
    return SELL_OK;
}

int check_matrix(const sell_mat *A) {
    if (!A) return SELL_ERR_ARG;
    if (!A->on_device) return SELL_ERR_STATE;
    int cur = -1;
    HIPCHK(hipGetDevice(&cur));
    return cur == A->device ? SELL_OK : SELL_ERR_STATE;
}

// Stream-ordered temporaries, released in stream order.
struct Temps {
    hipStream_t s;
    std::vector<void *> ptrs;
    explicit Temps(hipStream_t st) : s(st) {}
    ~Temps() {
        for (void *p : ptrs) (void)lib_free_async(p, s);
    }
    int alloc(void **p, size_t bytes) {
        *p = nullptr;
        HIPCHK(lib_malloc_async(p, bytes ? bytes : 16, s));
        ptrs.push_back(*p);
        return SELL_OK;
    }
};

sell_bv block(void *p, int64_t n, int b, int dt) {
    sell_bv v;
    v.nrows = n;
    v.ncols = b;
    v.dt = dt;
    v.lay = SELL_ROW_MAJOR;
    v.ptr = p;
    v.ld = b;
    v.owned = false;
    return v;
}

// y <- alpha (M x - c x) + beta y  (beta == 0: y not read)
int shifted_product(const sell_mat *M, const sell_bv &x, sell_bv &y, double alpha, double c, double beta,
                    hipStream_t s) {
    sell_spmv_opts o = SELL_SPMV_OPTS_INIT;
    o.flags = SELL_SPMV_SCALE | SELL_SPMV_SHIFT | (beta != 0.0 ? SELL_SPMV_AXPBY : 0u);
    o.alpha = alpha;
    o.gamma = c;
    o.beta = beta;
    return aug_impl(M, &x, &y, nullptr, o, true, s);
}

}  // namespace

extern "C" {

int sell_grad_values(const sell_mat *A, const sell_bv *G, const sell_bv *X, double alpha, int accumulate,
                     double *dval, void *stream) {
    int rc = check_matrix(A);
    if (rc) return rc;
    if (!G || !X) return SELL_ERR_ARG;
    const int b = G->ncols;
    if ((rc = check_block(A, G, A->h.nrows, b)) || (rc = check_block(A, X, A->h.ncols, b))) return rc;
    if (!dval && A->h.nnz > 0) return SELL_ERR_ARG;
    if (A->h.nnz == 0) return SELL_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = ensure_update_maps(const_cast<sell_mat *>(A), s))) return rc;
    Temps T(s);
    double *dsell = nullptr;
    if ((rc = T.alloc(reinterpret_cast<void **>(&dsell), size_t(A->h.stored) * sizeof(double)))) return rc;
    if ((rc = launch_fill(dsell, SELL_F64, A->h.stored, 1, 1, 1, 0.0, s))) return rc;
    if ((rc = launch_grad_accum(A, G->ptr, G->ld, X->ptr, X->ld, G->dt, b, alpha, dsell, s))) return rc;
    return launch_sell_to_csr(A, dsell, accumulate ? 1 : 0, dval, s);
}

int sell_cheb_forward(const sell_mat *A, const sell_bv *X, sell_bv *Y, int64_t N, double scale, double c,
                      int64_t K, void *ckpt, void *stream) {
    int rc = check_matrix(A);
    if (rc) return rc;
    if (A->h.nrows != A->h.ncols) return SELL_ERR_SHAPE;
    if (!X || !Y) return SELL_ERR_ARG;
    const int64_t n = A->h.nrows;
    const int b = X->ncols;
    if ((rc = check_block(A, X, n, b)) || (rc = check_block(A, Y, n, b))) return rc;
    if (b > kMaxSliceCols) return SELL_ERR_UNSUPPORTED;
    if (N < 1 || K < 1 || !(scale != 0.0) || !std::isfinite(scale) || !std::isfinite(c)) return SELL_ERR_ARG;
    if (n == 0) return SELL_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int dt = vec_dt_of(A);
    const size_t vb = size_t(n) * b * (dt == SELL_F64 ? 8 : 4);
    Temps T(s);
    void *p0, *p1;
    if ((rc = T.alloc(&p0, vb)) || (rc = T.alloc(&p1, vb))) return rc;
    sell_bv V0 = block(p0, n, b, dt), V1 = block(p1, n, b, dt);
    char *ck = static_cast<char *>(ckpt);
    if ((rc = launch_copy(&V0, X, s))) return rc;
    if ((rc = shifted_product(A, V0, V1, 1.0 / scale, c, 0.0, s))) return rc;  // v1 = A~ v0
    auto save = [&](int64_t k) -> int {
        if (!ck) return SELL_OK;
        HIPCHK(hipMemcpyAsync(ck + size_t(2 * k) * vb, V0.ptr, vb, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(ck + size_t(2 * k + 1) * vb, V1.ptr, vb, hipMemcpyDeviceToDevice, s));
        return SELL_OK;
    };
    if ((rc = save(0))) return rc;
    for (int64_t m = 1; m < N; ++m) {
        // v_m+1 = 2 A~ v_m - v_m-1, written over v_m-1
        if ((rc = shifted_product(A, V1, V0, 2.0 / scale, c, -1.0, s))) return rc;
        std::swap(V0, V1);  // (V0, V1) = (v_m, v_m+1)
        if (m % K == 0 && (rc = save(m / K))) return rc;
    }
    return launch_copy(Y, &V1, s);
}

int sell_cheb_filter(const sell_mat *A, const sell_bv *X, sell_bv *Z, int64_t N, const double *coef, double scale,
                     double c, void *stream) {
    int rc = check_matrix(A);
    if (rc) return rc;
    if (A->h.nrows != A->h.ncols) return SELL_ERR_SHAPE;
    if (!X || !Z || !coef) return SELL_ERR_ARG;
    const int64_t n = A->h.nrows;
    const int b = X->ncols;
    if ((rc = check_block(A, X, n, b)) || (rc = check_block(A, Z, n, b))) return rc;
    if (b > kMaxSliceCols) return SELL_ERR_UNSUPPORTED;
    if (N < 0 || !(scale != 0.0) || !std::isfinite(scale) || !std::isfinite(c)) return SELL_ERR_ARG;
    if (X->ptr == Z->ptr && n > 0) return SELL_ERR_ARG;
    if (n == 0) return SELL_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int dt = vec_dt_of(A);
    // z = coef_0 x
    if ((rc = launch_axpby(dt, n, b, b, coef[0], X->ptr, 0.0, Z->ptr, s))) return rc;
    if (N == 0) return SELL_OK;
    const size_t vb = size_t(n) * b * (dt == SELL_F64 ? 8 : 4);
    Temps T(s);
    void *p0, *p1;
    if ((rc = T.alloc(&p0, vb)) || (rc = T.alloc(&p1, vb))) return rc;
    sell_bv V0 = block(p0, n, b, dt), V1 = block(p1, n, b, dt);
    if ((rc = launch_copy(&V0, X, s))) return rc;
    // every step: one augmented product forming v_m+1 with the chained z = z + coef_m+1 v_m+1
    sell_spmv_opts o = SELL_SPMV_OPTS_INIT;
    o.flags = SELL_SPMV_SCALE | SELL_SPMV_SHIFT | SELL_SPMV_CHAIN;
    o.alpha = 1.0 / scale;
    o.gamma = c;
    o.delta = 1.0;
    o.eta = coef[1];
    if ((rc = aug_impl(A, &V0, &V1, Z, o, true, s))) return rc;  // v_1 = A~ v_0
    o.flags |= SELL_SPMV_AXPBY;
    o.alpha = 2.0 / scale;
    o.beta = -1.0;
    for (int64_t m = 1; m < N; ++m) {
        // v_m+1 = 2 A~ v_m - v_m-1, written over v_m-1
        o.eta = coef[m + 1];
        if ((rc = aug_impl(A, &V1, &V0, Z, o, true, s))) return rc;
        std::swap(V0, V1);  // (V0, V1) = (v_m, v_m+1)
    }
    return SELL_OK;
}

int sell_cheb_backward(const sell_mat *A, const sell_bv *G, int64_t N, double scale, double c, int64_t K,
                       const void *ckpt, sell_bv *dX, double *dval, void *stream) {
    int rc = check_matrix(A);
    if (rc) return rc;
    if (A->h.nrows != A->h.ncols) return SELL_ERR_SHAPE;
    if (!G || !dX || !ckpt) return SELL_ERR_ARG;
    const int64_t n = A->h.nrows;
    const int b = G->ncols;
    if ((rc = check_block(A, G, n, b)) || (rc = check_block(A, dX, n, b))) return rc;
    if (b > kMaxSliceCols) return SELL_ERR_UNSUPPORTED;
    if (N < 1 || K < 1 || !(scale != 0.0) || !std::isfinite(scale) || !std::isfinite(c)) return SELL_ERR_ARG;
    if (!dval && A->h.nnz > 0) return SELL_ERR_ARG;
    if (n == 0) return SELL_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    try {
        if ((rc = ensure_transpose(A, s)) || (rc = ensure_update_maps(const_cast<sell_mat *>(A), s))) return rc;
    } catch (const std::bad_alloc &) {
        return SELL_ERR_OOM;
    }
    const sell_mat *AT = A->transpose;
    const int dt = vec_dt_of(A);
    const size_t vb = size_t(n) * b * (dt == SELL_F64 ? 8 : 4);
    const int64_t nseg = (N + K - 1) / K;
    const int64_t seglen = std::min<int64_t>(K, N);
    Temps T(s);
    void *pw0, *pw1, *pwn, *pseg;
    double *dsell = nullptr;
    if ((rc = T.alloc(&pw0, vb)) || (rc = T.alloc(&pw1, vb)) || (rc = T.alloc(&pwn, vb)) ||
        (rc = T.alloc(&pseg, vb * size_t(seglen))) ||
        (rc = T.alloc(reinterpret_cast<void **>(&dsell), size_t(A->h.stored > 0 ? A->h.stored : 1) * 8)))
        return rc;
    sell_bv W1 = block(pw1, n, b, dt), W0 = block(pw0, n, b, dt), Wn = block(pwn, n, b, dt);
    auto seg = [&](int64_t i) { return block(static_cast<char *>(pseg) + size_t(i) * vb, n, b, dt); };
    const char *ck = static_cast<const char *>(ckpt);
    if ((rc = launch_copy(&W1, G, s))) return rc;  // w_N = G
    if ((rc = launch_fill(W0.ptr, dt, n, b, b, 1, 0.0, s))) return rc;  // w_N-1 (partial) = 0
    if ((rc = launch_fill(dsell, SELL_F64, A->h.stored, 1, 1, 1, 0.0, s))) return rc;
    for (int64_t k = nseg - 1; k >= 0; --k) {
        const int64_t lo = k * K, hi = std::min(lo + K - 1, N - 1);
        // recompute v_lo .. v_hi of this segment from its checkpoint (v_lo, v_lo+1)
        HIPCHK(hipMemcpyAsync(seg(0).ptr, ck + size_t(2 * k) * vb, vb, hipMemcpyDeviceToDevice, s));
        if (hi > lo) HIPCHK(hipMemcpyAsync(seg(1).ptr, ck + size_t(2 * k + 1) * vb, vb, hipMemcpyDeviceToDevice, s));
        for (int64_t m = lo + 2; m <= hi; ++m) {
            sell_bv prev = seg(m - lo - 1), out = seg(m - lo), prev2 = seg(m - lo - 2);
            if ((rc = launch_copy(&out, &prev2, s))) return rc;
            if ((rc = shifted_product(A, prev, out, 2.0 / scale, c, -1.0, s))) return rc;
        }
        for (int64_t m = hi; m >= std::max<int64_t>(lo, 1); --m) {
            // W1 = w_m+1 (complete), W0 = w_m (partial)
            sell_bv vm = seg(m - lo);
            if ((rc = launch_grad_accum(A, W1.ptr, b, vm.ptr, b, dt, b, 2.0 / scale, dsell, s))) return rc;
            if ((rc = launch_axpby(dt, n, b, b, -1.0, W1.ptr, 0.0, Wn.ptr, s))) return rc;  // w_m-1 = -w_m+1
            if ((rc = shifted_product(AT, W1, W0, 2.0 / scale, c, 1.0, s))) return rc;      // w_m += 2 A~^T w_m+1
            sell_bv t = W1;
            W1 = W0;
            W0 = Wn;
            Wn = t;
        }
        if (lo == 0) {
            // first step v_1 = A~ v_0: W1 = w_1, W0 = w_0 (partial)
            sell_bv v0 = seg(0);
            if ((rc = launch_grad_accum(A, W1.ptr, b, v0.ptr, b, dt, b, 1.0 / scale, dsell, s))) return rc;
            if ((rc = shifted_product(AT, W1, W0, 1.0 / scale, c, 1.0, s))) return rc;
        }
    }
    if ((rc = launch_copy(dX, &W0, s))) return rc;
    if (A->h.nnz == 0) return SELL_OK;
    return launch_sell_to_csr(A, dsell, 0, dval, s);
}

}  // extern "C"
