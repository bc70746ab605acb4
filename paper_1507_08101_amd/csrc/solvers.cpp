// solvers.cpp -- conjugate-gradient drivers on top of the augmented SpMMV.
//
// Both drivers run one CG per column of a block of right-hand sides (the paper's block
// vectors, Sec. 5.2, with per-column scalars as in its vaxpy/vaxpby operations). An
// iteration is one product and one vector pass, with no host synchronisation:
//   q = A p            augmented product with the fused dots <p, q> and <q, q>
//   alpha, beta        per-column scalars (device FP64); beta from <r', r'> = alpha^2 <q, q> - rho,
//                      which holds because q is A-orthogonal to the previous direction
//   r -= a q, x += a p, p = r + b p   the whole vector update in one pass, with <r, r>
// The host reads the per-column "active" flags every few iterations.
//
// sell_cg:        FP64 throughout; convergence is confirmed on the true residual b - A x.
// sell_cg_mixed:  FP64 iterative refinement by reliable updates. CG runs with FP32 vectors on
//                 the FP32 or BF16 matrix and accumulates its correction d in FP32; whenever
//                 the FP32 residual has dropped by inner_tol (or after inner_maxit steps) the
//                 correction is folded into x in FP64 and the residual is replaced by the
//                 true r = b - A x, formed in FP64 with the FP64 matrix (one augmented product:
//                 y = b preloaded, alpha = -1, beta = 1, fused <r, r>). The search direction is
//                 kept across updates, so the Krylov space is not restarted, unless the FP32
//                 recursion has drifted away from the true residual (its residual norm below a
//                 tenth of the true one, as when FP32 CG has exhausted a small system): then that
//                 column restarts from p = r, since the kept direction no longer fits the new r.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

using namespace sellcs;

namespace {

#define HIPCHK(x)                                                                      \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) return e_ == hipErrorOutOfMemory ? SELL_ERR_OOM : SELL_ERR_HIP; \
    } while (0)

constexpr int kCheckEvery = 8;

struct Buffers {
    std::vector<void *> ptrs;
    ~Buffers() {
        for (void *p : ptrs) lib_free(p);
    }
    int alloc(void **p, size_t bytes) {
        *p = nullptr;
        if (bytes == 0) bytes = 16;
        HIPCHK(lib_malloc(p, bytes));
        ptrs.push_back(*p);
        return SELL_OK;
    }
};

sell_bv view(void *p, int64_t n, int b, int dt) {
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

struct Scalars {
    double *rho, *pq, *alpha, *beta, *thresh2, *bb, *rr, *thresh_out;
    int32_t *active;
    int32_t *colmask;     // per-column flags handed to the device (b)
    double *prod_parts;   // tile partials of the product's dots (3 b ntiles)
    double *vec_parts;    // workgroup partials of the vector kernels (b kCgMaxGrid)
    int32_t prod_tiles;
    CgDev dev() const { return CgDev{rho, pq, alpha, beta, thresh2, active}; }
};

int alloc_scalars(Buffers &B, Scalars &S, int b, int32_t max_tiles) {
    double *d = nullptr;
    const size_t nt = size_t(max_tiles > 0 ? max_tiles : 1);
    const size_t n = 16 * size_t(b) + 3 * size_t(b) * nt + size_t(b) * kCgMaxGrid + 64;
    int rc = B.alloc(reinterpret_cast<void **>(&d), sizeof(double) * n);
    if (rc) return rc;
    S.rho = d;
    S.pq = d + b;
    S.alpha = d + 2 * b;
    S.beta = d + 3 * b;
    S.thresh2 = d + 4 * b;
    S.bb = d + 5 * b;
    S.rr = d + 6 * b;         // 3b
    S.thresh_out = d + 9 * b;
    S.active = reinterpret_cast<int32_t *>(d + 11 * b);
    S.colmask = reinterpret_cast<int32_t *>(d + 13 * b);
    S.prod_parts = d + 16 * b;
    S.vec_parts = S.prod_parts + 3 * size_t(b) * nt;
    S.prod_tiles = max_tiles;
    return SELL_OK;
}

int any_active(const Scalars &S, int b, hipStream_t s, bool *any) {
    int32_t h[64];
    HIPCHK(hipMemcpyAsync(h, S.active, sizeof(int32_t) * b, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *any = false;
    for (int j = 0; j < b; ++j) *any = *any || h[j] != 0;
    return SELL_OK;
}

// CG iterations on A for X (correction or solution), R (current residual), P, Q work.
// Expects S.rho, S.thresh2 and S.active set for R. Runs until no column is active or
// maxit iterations; returns the iterations done in *its.
int cg_iterate(const sell_mat *A, int dt, sell_bv &X, sell_bv &R, sell_bv &P, sell_bv &Q, const Scalars &S,
               int64_t maxit, int64_t *its, hipStream_t s) {
    const int64_t n = A->h.nrows;
    const int b = R.ncols;
    int rc = launch_copy(&P, &R, s);
    if (rc) return rc;
    sell_spmv_opts o = SELL_SPMV_OPTS_INIT;
    o.flags = SELL_SPMV_DOT_XY | SELL_SPMV_DOT_YY;
    *its = 0;
    bool any = true;
    if ((rc = any_active(S, b, s, &any))) return rc;
    while (any && *its < maxit) {
        int32_t nblk = 0;
        if ((rc = aug_impl(A, &P, &Q, nullptr, o, true, s, S.prod_parts, &nblk))) return rc;
        if ((rc = cg_launch_step(S.prod_parts, nblk, b, S.dev(), s))) return rc;
        if ((rc = cg_launch_rp(dt, R.ptr, Q.ptr, P.ptr, X.ptr, n, b, b, S.dev(), S.vec_parts, s))) return rc;
        ++*its;
        if (*its % kCheckEvery == 0 && (rc = any_active(S, b, s, &any))) return rc;
    }
    return SELL_OK;
}

// r = b - A x in FP64 (b preloaded into R), <r, r> into S.rr[0..b)
int true_residual(const sell_mat *A64, const sell_bv *Bv, const sell_bv *X, sell_bv &R, const Scalars &S,
                  hipStream_t s) {
    int rc = launch_copy(&R, Bv, s);
    if (rc) return rc;
    sell_spmv_opts o = SELL_SPMV_OPTS_INIT;
    o.flags = SELL_SPMV_SCALE | SELL_SPMV_AXPBY | SELL_SPMV_DOT_YY;
    o.alpha = -1.0;
    o.beta = 1.0;
    o.dot = S.rr;
    return aug_impl(A64, X, &R, nullptr, o, true, s);
}

int relres_host(const Scalars &S, int b, hipStream_t s, double *worst) {
    double rr[64], bb[64];
    HIPCHK(hipMemcpyAsync(rr, S.rr, sizeof(double) * b, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(bb, S.bb, sizeof(double) * b, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *worst = 0.0;
    for (int j = 0; j < b; ++j) {
        const double r = bb[j] > 0 ? std::sqrt(rr[j] / bb[j]) : std::sqrt(rr[j]);
        if (!(r <= *worst)) *worst = r;  // NaN propagates
    }
    return SELL_OK;
}

int check_cg_operands(const sell_mat *A, const sell_bv *Bv, const sell_bv *X) {
    if (!A || !Bv || !X) return SELL_ERR_ARG;
    if (!A->on_device) return SELL_ERR_STATE;
    if (A->h.nrows != A->h.ncols) return SELL_ERR_SHAPE;
    if (Bv->dt != SELL_F64 || X->dt != SELL_F64) return SELL_ERR_DTYPE;
    if (Bv->nrows != A->h.nrows || X->nrows != A->h.nrows || Bv->ncols != X->ncols) return SELL_ERR_SHAPE;
    if (Bv->ncols < 1 || Bv->ncols > 64) return SELL_ERR_UNSUPPORTED;
    if (Bv->lay != SELL_ROW_MAJOR || X->lay != SELL_ROW_MAJOR || Bv->ld != Bv->ncols || X->ld != X->ncols)
        return SELL_ERR_UNSUPPORTED;
    if ((!Bv->ptr || !X->ptr) && A->h.nrows > 0) return SELL_ERR_ARG;
    return SELL_OK;
}

}  // namespace

extern "C" {

int sell_cg(const sell_mat *A, const sell_bv *Bv, sell_bv *X, double tol, int64_t maxit, sell_cg_stats *stats,
            void *stream) {
    int rc = check_cg_operands(A, Bv, X);
    if (rc) return rc;
    if (A->h.vdt != SELL_F64) return SELL_ERR_DTYPE;
    if (!(tol > 0) || maxit < 0) return SELL_ERR_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = A->h.nrows;
    const int b = Bv->ncols;
    sell_cg_stats st{0, 0, 0.0, 0};
    if (n == 0) {
        st.converged = 1;
        if (stats) *stats = st;
        return SELL_OK;
    }
    Buffers B;
    void *pr, *pp, *pq;
    const size_t bytes = size_t(n) * b * sizeof(double);
    if ((rc = B.alloc(&pr, bytes)) || (rc = B.alloc(&pp, bytes)) || (rc = B.alloc(&pq, bytes))) return rc;
    Scalars S;
    if ((rc = alloc_scalars(B, S, b, A->ntiles))) return rc;
    sell_bv R = view(pr, n, b, SELL_F64), P = view(pp, n, b, SELL_F64), Q = view(pq, n, b, SELL_F64);
    // ||b||^2 and the stopping threshold tol^2 ||b||^2
    if ((rc = cg_launch_coldot(SELL_F64, Bv->ptr, Bv->ptr, n, b, b, S.bb, S.vec_parts, S.thresh_out,
                               S.active, nullptr, tol * tol, s)))
        return rc;
    double worst = 0.0;
    while (true) {
        if ((rc = true_residual(A, Bv, X, R, S, s))) return rc;
        if ((rc = relres_host(S, b, s, &worst))) return rc;
        if (worst <= tol || st.iterations >= maxit) break;
        // rho = <r, r>, active = rho > tol^2 ||b||^2
        if ((rc = cg_launch_coldot(SELL_F64, R.ptr, R.ptr, n, b, b, S.rho, S.vec_parts, S.thresh2,
                                   S.active, S.thresh_out, 1.0, s)))
            return rc;
        int64_t its = 0;
        if ((rc = cg_iterate(A, SELL_F64, *X, R, P, Q, S, maxit - st.iterations, &its, s))) return rc;
        st.iterations += its;
        if (its == 0) break;
        ++st.refinements;  // restarts from the true residual
    }
    st.refinements = st.refinements > 0 ? st.refinements - 1 : 0;
    st.relres = worst;
    st.converged = worst <= tol ? 1 : 0;
    if (stats) *stats = st;
    return SELL_OK;
}

int sell_cg_mixed(const sell_mat *A64, const sell_mat *Alo, const sell_bv *Bv, sell_bv *X, double tol,
                  int64_t maxit, double inner_tol, int64_t inner_maxit, sell_cg_stats *stats, void *stream) {
    int rc = check_cg_operands(A64, Bv, X);
    if (rc) return rc;
    if (!Alo) return SELL_ERR_ARG;
    if (!Alo->on_device) return SELL_ERR_STATE;
    if (A64->h.vdt != SELL_F64 || Alo->h.vdt == SELL_F64) return SELL_ERR_DTYPE;
    if (Alo->h.nrows != A64->h.nrows || Alo->h.ncols != A64->h.ncols || Alo->h.nnz != A64->h.nnz)
        return SELL_ERR_SHAPE;
    if (!(tol > 0) || !(inner_tol > 0) || !(inner_tol < 1) || maxit < 0 || inner_maxit < 1) return SELL_ERR_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = A64->h.nrows;
    const int b = Bv->ncols;
    sell_cg_stats st{0, 0, 0.0, 0};
    if (n == 0) {
        st.converged = 1;
        if (stats) *stats = st;
        return SELL_OK;
    }
    Buffers B;
    void *pr64, *pr, *pd, *pp, *pq;
    const size_t b64 = size_t(n) * b * sizeof(double), b32 = size_t(n) * b * sizeof(float);
    if ((rc = B.alloc(&pr64, b64)) || (rc = B.alloc(&pr, b32)) || (rc = B.alloc(&pd, b32)) ||
        (rc = B.alloc(&pp, b32)) || (rc = B.alloc(&pq, b32)))
        return rc;
    Scalars S;
    if ((rc = alloc_scalars(B, S, b, std::max(A64->ntiles, Alo->ntiles)))) return rc;
    sell_bv R64 = view(pr64, n, b, SELL_F64);
    sell_bv R = view(pr, n, b, SELL_F32), D = view(pd, n, b, SELL_F32), P = view(pp, n, b, SELL_F32),
            Q = view(pq, n, b, SELL_F32);
    // ||b||^2 (into S.bb)
    if ((rc = cg_launch_coldot(SELL_F64, Bv->ptr, Bv->ptr, n, b, b, S.bb, S.vec_parts, nullptr, nullptr, nullptr,
                               0.0, s)))
        return rc;
    double bb[64], rr[64], rho[64], rho_last[64];
    int32_t act[64], reset[64];
    for (int j = 0; j < b; ++j) rho[j] = 0.0;
    HIPCHK(hipMemcpyAsync(bb, S.bb, sizeof(double) * b, hipMemcpyDeviceToHost, s));

    // Reliable update: fold the FP32 correction into x (FP64), recompute the true residual
    // r = b - A x in FP64, restart the FP32 recursion from it (the search direction is
    // kept). Returns through *done whether every column meets the tolerance.
    auto reliable_update = [&](bool fold, bool *done) -> int {
        int r;
        if (fold && (r = cg_launch_axpy_mixed(static_cast<double *>(X->ptr), static_cast<const float *>(D.ptr), n,
                                              b, b, s)))
            return r;
        if ((r = true_residual(A64, Bv, X, R64, S, s))) return r;
        HIPCHK(hipMemcpyAsync(rr, S.rr, sizeof(double) * b, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        double worst = 0.0;
        bool all = true;
        for (int j = 0; j < b; ++j) {
            const double rel = bb[j] > 0 ? std::sqrt(rr[j] / bb[j]) : std::sqrt(rr[j]);
            if (!(rel <= worst)) worst = rel;
            act[j] = rel <= tol ? 0 : 1;
            all = all && !act[j];
        }
        st.relres = worst;
        *done = all;
        if (all) return SELL_OK;
        bool any_reset = false;
        for (int j = 0; j < b; ++j) {
            reset[j] = (act[j] && !(rho[j] >= 0.01 * rr[j])) ? 1 : 0;  // recursion drifted (or first update)
            any_reset = any_reset || reset[j];
        }
        if ((r = launch_copy(&R, &R64, s))) return r;  // FP64 -> FP32, round to nearest
        if ((r = launch_fill(D.ptr, SELL_F32, n, b, b, 1, 0.0, s))) return r;
        // rho = <r32, r32>; thresh2 = 0 so the FP32 recursion never retires a column itself
        if ((r = cg_launch_coldot(SELL_F32, R.ptr, R.ptr, n, b, b, S.rho, S.vec_parts, S.thresh2, S.active, nullptr,
                                  0.0, s)))
            return r;
        HIPCHK(hipMemcpyAsync(S.active, act, sizeof(int32_t) * b, hipMemcpyHostToDevice, s));
        if (any_reset) {
            HIPCHK(hipMemcpyAsync(S.colmask, reset, sizeof(int32_t) * b, hipMemcpyHostToDevice, s));
            if ((r = cg_launch_copy_cols(SELL_F32, P.ptr, R.ptr, n, b, b, S.colmask, s))) return r;
        }
        HIPCHK(hipMemcpyAsync(rho_last, S.rho, sizeof(double) * b, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int j = 0; j < b; ++j) rho[j] = rho_last[j];
        return SELL_OK;
    };

    bool done = false;
    // p = 0 in every column (a converged column keeps it); the first update sets p = r in the
    // active columns (rho = 0 there marks the recursion as drifted)
    if ((rc = launch_fill(P.ptr, SELL_F32, n, b, b, 1, 0.0, s))) return rc;
    if ((rc = reliable_update(false, &done))) return rc;
    sell_spmv_opts o = SELL_SPMV_OPTS_INIT;
    o.flags = SELL_SPMV_DOT_XY | SELL_SPMV_DOT_YY;
    int64_t since = 0;
    while (!done && st.iterations < maxit) {
        int32_t nblk = 0;
        if ((rc = aug_impl(Alo, &P, &Q, nullptr, o, true, s, S.prod_parts, &nblk))) return rc;
        if ((rc = cg_launch_step(S.prod_parts, nblk, b, S.dev(), s))) return rc;
        if ((rc = cg_launch_rp(SELL_F32, R.ptr, Q.ptr, P.ptr, D.ptr, n, b, b, S.dev(), S.vec_parts, s))) return rc;
        ++st.iterations;
        ++since;
        if (st.iterations % kCheckEvery == 0 || st.iterations == maxit) {
            HIPCHK(hipMemcpyAsync(rho, S.rho, sizeof(double) * b, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            bool update = st.iterations == maxit || since >= inner_maxit;
            for (int j = 0; j < b; ++j)
                if (act[j] && (!(rho[j] > inner_tol * inner_tol * rho_last[j]))) update = true;  // NaN too
            if (update) {
                if ((rc = reliable_update(true, &done))) return rc;
                ++st.refinements;
                since = 0;
            }
        }
    }
    if (!done && st.iterations > 0 && since > 0) {
        if ((rc = reliable_update(true, &done))) return rc;
        ++st.refinements;
    }
    st.converged = done ? 1 : 0;
    if (stats) *stats = st;
    return SELL_OK;
}

}  // extern "C"
