// batch_solve.cpp -- conjugate gradients for a batch of independent systems, all of them
// advanced by the same kernel launches.
//
// Every system m (matrix A_m of the batch, right-hand sides B_m, one CG per column) keeps its
// own FP64 scalars on the device. One iteration over the whole batch is four launches:
//   Q = A P            batched product with the fused <p, q> and <q, q> per system and column
//   alpha, beta        one workgroup per system (beta from <r', r'> = alpha^2 <q, q> - rho)
//   R -= a Q, D += a P, P = R + b P   one segmented vector pass with the partials of <r, r>
//   rho, flags         one workgroup per system (a system whose columns have all converged
//                      drops out: the product and vector kernels skip it)
// Runs of kCheckEvery iterations are captured in a HIP graph and replayed (or launched
// directly); the host looks at the scalars between runs. The launches of an iteration are
// spread over the systems that still iterate only: whenever that set changes, the resident
// workgroups of the product and of the vector kernels are split anew over the remaining
// systems (and the graph is captured again), so that the last, largest systems still get the
// whole GPU. A residual update likewise spreads its FP64 product over the updated systems.
//
// Precision: with a low-precision batch Alo (F32 or BF16 values) the iteration runs in FP32
// vectors and accumulates a correction D, and the solution is refined in FP64 by reliable
// updates per system: when the FP32 residual of one of the system's columns has dropped by
// inner_tol since the system's last update (or after inner_maxit iterations), D is folded into
// x in FP64 and the residual replaced by the true r = b - A64 x, computed in FP64 with the F64
// matrix. Without Alo the iteration runs in FP64 on A64; a system's columns retire when their
// recursive residual meets the tolerance and the true residual then confirms them (or
// restarts the system from it). In both cases the search direction is kept across updates,
// except in a column whose recursive residual has drifted below a tenth of the true one (FP32
// CG that has exhausted a small system, or a retired column): the kept direction no longer
// fits the new residual there, and the column restarts from p = r.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

using namespace sellcs;

namespace sellcs {
int batch_aug_impl(sell_batch *B, const sell_bv *X, sell_bv *Y, sell_bv *Z, const sell_spmv_opts &o, bool aug,
                   const int32_t *active, const int32_t *host_active, bool finish, hipStream_t s,
                   const int32_t **out_blk, const double **out_partials, bool reserved);
void apportion(const std::vector<double> &w, const std::vector<int64_t> &cap, int32_t G0,
               std::vector<int32_t> &blk);
const sell_mat *batch_matrix(const sell_batch *B, int m);
int32_t batch_count(const sell_batch *B);
int64_t batch_rows(const sell_batch *B);
int batch_vdt(const sell_batch *B);
BatchSeg batch_seg(const sell_batch *B);
bool batch_ragged(const sell_batch *B, int b);
}  // namespace sellcs

namespace {

#define HIPCHK(x)                                                                             \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess) return e_ == hipErrorOutOfMemory ? SELL_ERR_OOM : SELL_ERR_HIP; \
    } while (0)

constexpr int kCheckEvery = 8;

struct DevBuffers {
    std::vector<void *> ptrs;
    ~DevBuffers() {
        for (void *p : ptrs) (void)lib_free(p);
    }
    int alloc(void **p, size_t bytes) {
        *p = nullptr;
        if (bytes == 0) bytes = 16;
        HIPCHK(lib_malloc(p, bytes));
        ptrs.push_back(*p);
        return SELL_OK;
    }
};

struct OwnedStream {
    hipStream_t s = nullptr;
    bool owned = false;
    ~OwnedStream() {
        if (owned) {
            (void)hipStreamSynchronize(s);
            drop_workspace(s);
            (void)hipStreamDestroy(s);
        }
    }
};

struct Graph {
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    ~Graph() {
        if (ge) (void)hipGraphExecDestroy(ge);
        if (g) (void)hipGraphDestroy(g);
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

int check_batches(sell_batch *A64, sell_batch *Alo, const sell_bv *Bv, const sell_bv *X) {
    if (!A64 || !Bv || !X) return SELL_ERR_ARG;
    if (batch_vdt(A64) != SELL_F64) return SELL_ERR_DTYPE;
    const int K = batch_count(A64);
    for (int m = 0; m < K; ++m) {
        const sell_mat *A = batch_matrix(A64, m);
        int rc = check_device(A);
        if (rc) return rc;
        if (A->h.nrows != A->h.ncols) return SELL_ERR_SHAPE;
    }
    if (Alo) {
        if (batch_vdt(Alo) == SELL_F64) return SELL_ERR_DTYPE;
        if (batch_count(Alo) != K) return SELL_ERR_SHAPE;
        for (int m = 0; m < K; ++m) {
            const sell_mat *A = batch_matrix(A64, m), *L = batch_matrix(Alo, m);
            int rc = check_device(L);
            if (rc) return rc;
            if (L->h.nrows != A->h.nrows || L->h.ncols != A->h.ncols || L->h.nnz != A->h.nnz) return SELL_ERR_SHAPE;
        }
    }
    if (Bv->dt != SELL_F64 || X->dt != SELL_F64) return SELL_ERR_DTYPE;
    const int64_t n = batch_rows(A64);
    if (Bv->nrows != n || X->nrows != n || Bv->ncols != X->ncols) return SELL_ERR_SHAPE;
    if (Bv->ncols < 1 || Bv->ncols > 64) return SELL_ERR_UNSUPPORTED;
    if (Bv->lay != SELL_ROW_MAJOR || X->lay != SELL_ROW_MAJOR || Bv->ld != Bv->ncols || X->ld != X->ncols)
        return SELL_ERR_UNSUPPORTED;
    if ((!Bv->ptr || !X->ptr) && n > 0) return SELL_ERR_ARG;
    return SELL_OK;
}

}  // namespace

extern "C" {

int sell_batch_cg(sell_batch *A64, sell_batch *Alo, const sell_bv *Bv, sell_bv *X, double tol, int64_t maxit,
                  double inner_tol, int64_t inner_maxit, uint32_t flags, sell_cg_stats *stats, void *stream) {
    int rc = check_batches(A64, Alo, Bv, X);
    if (rc) return rc;
    const bool mixed = Alo != nullptr;
    if (!(tol > 0) || maxit < 0 || inner_maxit < 1) return SELL_ERR_ARG;
    if (mixed && !(inner_tol > 0 && inner_tol < 1)) return SELL_ERR_ARG;
    if (flags & ~uint32_t(SELL_BATCH_GRAPH)) return SELL_ERR_ARG;
    const bool use_graph = (flags & SELL_BATCH_GRAPH) != 0;
    const int K = batch_count(A64);
    const int b = Bv->ncols;
    if (batch_ragged(A64, b) || (mixed && batch_ragged(Alo, b))) return SELL_ERR_UNSUPPORTED;
    const int64_t n = batch_rows(A64);
    const int idt = mixed ? SELL_F32 : SELL_F64;  // vector type of the iteration
    const size_t isz = mixed ? sizeof(float) : sizeof(double);
    sell_batch *Ain = mixed ? Alo : A64;
    const BatchSeg sg = batch_seg(A64);  // every system (for ||b||^2 and the residual updates)
    const size_t Kb = size_t(K) * b;
    if (n == 0) {  // only empty systems: nothing to solve
        if (stats)
            for (int m = 0; m < K; ++m) stats[m] = sell_cg_stats{0, 0, 0.0, 1};
        return SELL_OK;
    }

    // a stream of our own when the caller passes the legacy default stream (which cannot be
    // captured); created blocking, so it is ordered after the caller's earlier work
    OwnedStream os;
    os.s = static_cast<hipStream_t>(stream);
    if (!os.s) {
        HIPCHK(hipStreamCreate(&os.s));
        os.owned = true;
    }
    hipStream_t s = os.s;

    DevBuffers DB;
    void *pr64, *pr, *pd, *pp, *pq, *pscal;
    const size_t nv = size_t(n) * b;
    if ((rc = DB.alloc(&pr64, nv * sizeof(double))) || (rc = DB.alloc(&pr, nv * isz)) ||
        (rc = DB.alloc(&pd, nv * isz)) || (rc = DB.alloc(&pp, nv * isz)) || (rc = DB.alloc(&pq, nv * isz)))
        return rc;
    // device scalars: rho alpha beta thresh2 bb rr(3Kb) | vec partials (b G) | int32 flags
    // vector-kernel workgroups of an iteration (4,096 and 8,192 ran 1-2 % faster than 2,048 and
    // 1,024 with 8 rows in flight per thread)
    const int32_t Gv = 4 * kCgMaxGrid;
    const size_t gmax = size_t(std::max(std::max(sg.G, Gv), K));
    const size_t nd = 5 * Kb + 3 * Kb + size_t(b) * gmax;
    // active, sys_active, mask | iters (int64) | column mask | iteration and update workgroup offsets
    const size_t ni = Kb + 2 * size_t(K) + 2 * size_t(K) + 2 + Kb + 2 * (size_t(K) + 1);
    if ((rc = DB.alloc(&pscal, nd * sizeof(double) + ni * sizeof(int32_t) + 16)))
        return rc;
    double *d = static_cast<double *>(pscal);
    BatchCg sc;
    sc.rho = d;
    sc.alpha = d + Kb;
    sc.beta = d + 2 * Kb;
    sc.thresh2 = d + 3 * Kb;
    double *bb_d = d + 4 * Kb;
    double *rr_d = d + 5 * Kb;
    double *vparts = d + 8 * Kb;
    int32_t *ip = reinterpret_cast<int32_t *>(d + nd);
    sc.active = ip;
    sc.sys_active = ip + Kb;
    int32_t *mask_d = ip + Kb + K;
    int64_t *iters_d = reinterpret_cast<int64_t *>(ip + Kb + 2 * size_t(K));
    // align the int64 counters
    iters_d = reinterpret_cast<int64_t *>((reinterpret_cast<uintptr_t>(iters_d) + 7) & ~uintptr_t(7));
    sc.iters = iters_d;
    int32_t *colmask_d = reinterpret_cast<int32_t *>(iters_d + K);
    int32_t *vblk_d = colmask_d + Kb;
    int32_t *vblkr_d = vblk_d + K + 1;

    sell_bv Bview = *Bv;
    sell_bv R64 = view(pr64, n, b, SELL_F64), R = view(pr, n, b, idt), D = view(pd, n, b, idt),
            P = view(pp, n, b, idt), Q = view(pq, n, b, idt);
    if ((rc = launch_fill(pd, idt, n, b, b, 1, 0.0, s))) return rc;
    if ((rc = launch_fill(pp, idt, n, b, b, 1, 0.0, s))) return rc;
    if ((rc = launch_fill(iters_d, SELL_F64, 1, K, K, 1, 0.0, s))) return rc;  // all-zero bits
    // ||b||^2 per system and column
    if ((rc = bcg_launch_coldot(SELL_F64, Bv->ptr, Bv->ptr, b, sg, nullptr, vparts, bb_d, nullptr, nullptr, 0.0, s)))
        return rc;
    std::vector<double> bb(Kb), rr(3 * Kb), rho(Kb), rho_last(Kb, 0.0), relres(size_t(K), INFINITY);
    std::vector<int32_t> act(Kb, 1), sysact(size_t(K), 0), conv(size_t(K), 0), mask(size_t(K), 0), reset(Kb, 0);
    std::vector<int64_t> since(size_t(K), 0), refine(size_t(K), 0), its(size_t(K), 0);
    HIPCHK(hipMemcpyAsync(bb.data(), bb_d, Kb * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));

    std::vector<double> wrows(static_cast<size_t>(K));
    for (int m = 0; m < K; ++m) wrows[size_t(m)] = double(batch_matrix(A64, m)->h.nrows);
    // The workgroups of the update's vector kernels, split over the systems it updates (with the
    // batch's own split, an update of a few systems ran on their small share of the grid).
    std::vector<int32_t> vblkr;
    BatchSeg sgr = sg;
    sgr.vblk = vblkr_d;

    // Reliable update of the systems with mask[m] != 0: fold D into x, true residual in FP64,
    // restart the systems that have not converged from it.
    auto refresh = [&]() -> int {
        int r;
        HIPCHK(hipMemcpyAsync(mask_d, mask.data(), K * sizeof(int32_t), hipMemcpyHostToDevice, s));
        {
            std::vector<int64_t> cap(static_cast<size_t>(K));
            for (int m = 0; m < K; ++m) {
                const int64_t nr = batch_matrix(A64, m)->h.nrows;
                cap[size_t(m)] = (mask[size_t(m)] && nr > 0) ? std::max<int64_t>(1, (nr + 3) / 4) : 0;
            }
            apportion(wrows, cap, Gv, vblkr);
            sgr.G = vblkr[size_t(K)];
            // vblkr is not touched again before the synchronisation below
            HIPCHK(hipMemcpyAsync(vblkr_d, vblkr.data(), (size_t(K) + 1) * sizeof(int32_t), hipMemcpyHostToDevice,
                                  s));
        }
        if ((r = bcg_launch_refresh_prep(idt, static_cast<double *>(X->ptr), pd, static_cast<double *>(pr64),
                                         static_cast<const double *>(Bv->ptr), b, sgr, mask_d, s)))
            return r;
        sell_spmv_opts o = SELL_SPMV_OPTS_INIT;
        o.flags = SELL_SPMV_SCALE | SELL_SPMV_AXPBY | SELL_SPMV_DOT_YY;
        o.alpha = -1.0;
        o.beta = 1.0;
        o.dot = rr_d;
        if ((r = batch_aug_impl(A64, X, &R64, nullptr, o, true, mask_d, mask.data(), true, s, nullptr, nullptr, false)))
            return r;
        HIPCHK(hipMemcpyAsync(rr.data(), rr_d, 3 * Kb * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        bool restart = false;
        for (int m = 0; m < K; ++m) {
            if (!mask[size_t(m)]) continue;
            ++refine[size_t(m)];
            since[size_t(m)] = 0;
            double worst = 0.0;
            bool all = true;
            for (int j = 0; j < b; ++j) {
                const size_t q = size_t(m) * b + j;
                const double r2 = rr[size_t(m) * 3 * b + j];  // group <y, y> of matrix m
                const double rel = bb[q] > 0 ? std::sqrt(r2 / bb[q]) : std::sqrt(r2);
                if (!(rel <= worst)) worst = rel;  // NaN propagates
                act[q] = rel <= tol ? 0 : 1;
                all = all && !act[q];
            }
            relres[size_t(m)] = worst;
            conv[size_t(m)] = all ? 1 : 0;
            sysact[size_t(m)] = all ? 0 : 1;
            if (all) mask[size_t(m)] = 0;  // nothing to restart
            restart = restart || !all;
        }
        HIPCHK(hipMemcpyAsync(sc.active, act.data(), Kb * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(sc.sys_active, sysact.data(), K * sizeof(int32_t), hipMemcpyHostToDevice, s));
        if (!restart) return SELL_OK;
        // columns whose recursion drifted from the true residual restart from p = r (rho holds
        // the recursive residuals of the last check; 0 before the first iteration)
        bool any_reset = false;
        for (int m = 0; m < K; ++m)
            for (int j = 0; j < b; ++j) {
                const size_t q = size_t(m) * b + j;
                const double r2 = rr[size_t(m) * 3 * b + j];
                reset[q] = (mask[size_t(m)] && act[q] && !(rho[q] >= 0.01 * r2)) ? 1 : 0;
                any_reset = any_reset || reset[q];
            }
        HIPCHK(hipMemcpyAsync(mask_d, mask.data(), K * sizeof(int32_t), hipMemcpyHostToDevice, s));
        // r = r64 in the iteration's precision, rho = <r, r>; the recursion retires a column
        // itself only in FP64 (thresh2 = tol^2 ||b||^2), in FP32 only the true residual does
        if ((r = bcg_launch_convert(idt, pr, static_cast<const double *>(pr64), b, sgr, mask_d, vparts, sc.rho,
                                    sc.thresh2, bb_d, mixed ? 0.0 : tol * tol, s)))
            return r;
        if (any_reset) {
            HIPCHK(hipMemcpyAsync(colmask_d, reset.data(), Kb * sizeof(int32_t), hipMemcpyHostToDevice, s));
            if ((r = bcg_launch_copy(idt, pp, pr, b, sgr, colmask_d, s))) return r;
        }
        HIPCHK(hipMemcpyAsync(rho.data(), sc.rho, Kb * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int m = 0; m < K; ++m)
            if (mask[size_t(m)])
                for (int j = 0; j < b; ++j) rho_last[size_t(m) * b + j] = rho[size_t(m) * b + j];
        return SELL_OK;
    };

    // first update: every system, x0 = X (D = 0, P = 0); rho = 0 makes every active column
    // start from p = r
    std::fill(mask.begin(), mask.end(), 1);
    if ((rc = refresh())) return rc;

    // the split of an iteration's launches over the systems that iterate (appo_active)
    std::vector<int32_t> appo_active(static_cast<size_t>(K), -1), vblk;
    BatchSeg sgi = sg;
    sgi.vblk = vblk_d;
    auto resplit = [&](bool *changed) -> int {
        *changed = appo_active != sysact;
        if (!*changed) return SELL_OK;
        appo_active = sysact;
        std::vector<int64_t> cap(static_cast<size_t>(K));
        for (int m = 0; m < K; ++m) {
            const int64_t nr = batch_matrix(A64, m)->h.nrows;
            cap[size_t(m)] = (sysact[size_t(m)] && nr > 0) ? std::max<int64_t>(1, (nr + 3) / 4) : 0;
        }
        apportion(wrows, cap, Gv, vblk);
        sgi.G = vblk[size_t(K)];
        HIPCHK(hipMemcpyAsync(vblk_d, vblk.data(), (size_t(K) + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));  // vblk is reused by the next split
        return SELL_OK;
    };

    sell_spmv_opts po = SELL_SPMV_OPTS_INIT;
    po.flags = SELL_SPMV_DOT_XY | SELL_SPMV_DOT_YY;
    auto iteration = [&]() -> int {
        int r;
        const int32_t *pblk = nullptr;
        const double *pparts = nullptr;
        if ((r = batch_aug_impl(Ain, &P, &Q, nullptr, po, true, sc.sys_active, appo_active.data(), false, s, &pblk,
                                &pparts, true)))
            return r;
        if ((r = bcg_launch_step(pparts, pblk, K, b, sc, s))) return r;
        if (sgi.G == 0) return SELL_OK;
        return bcg_launch_rp(idt, pr, pq, pp, pd, b, sgi, sc, vparts, s);
    };

    Graph graph;
    bool done = std::all_of(conv.begin(), conv.end(), [](int32_t c) { return c != 0; });
    int64_t it = 0;
    // Runs since the split last changed. A split is captured in a graph only from its third run
    // on: the first run places the product's table on the device, and splits that change after
    // one or two runs (systems retiring at different iterations) would pay a capture and an
    // instantiation for one replay. On the 64 Laplacians at b = 8 the split changed 31 times in
    // 56 runs; capturing from the second run took 13 captures for 25 replays, and the BF16-value
    // solve ran 0.677 s against 0.667 s without a graph. With 64 equal systems (3 changes in 33
    // runs) the graph runs 0.218 s against 0.225 s.
    int stable = 0;
    std::vector<int32_t> act_now(Kb), sys_now(static_cast<size_t>(K));
    while (!done && it < maxit) {
        bool changed = false;
        if ((rc = resplit(&changed))) return rc;
        if (changed) {
            stable = 0;
            if (graph.ge) (void)hipGraphExecDestroy(graph.ge);
            if (graph.g) (void)hipGraphDestroy(graph.g);
            graph.ge = nullptr;
            graph.g = nullptr;
        }
        const int64_t run = std::min<int64_t>(kCheckEvery, maxit - it);
        if (use_graph && run == kCheckEvery && stable >= 2) {
            if (!graph.ge) {
                HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                int r = SELL_OK;
                for (int k = 0; k < run && r == SELL_OK; ++k) r = iteration();
                hipGraph_t g = nullptr;
                const hipError_t e = hipStreamEndCapture(s, &g);
                graph.g = g;
                if (r) return r;
                HIPCHK(e);
                HIPCHK(hipGraphInstantiate(&graph.ge, graph.g, nullptr, nullptr, 0));
            }
            HIPCHK(hipGraphLaunch(graph.ge, s));
        } else {
            for (int64_t k = 0; k < run; ++k)
                if ((rc = iteration())) return rc;
        }
        ++stable;
        it += run;
        for (int m = 0; m < K; ++m)
            if (sysact[size_t(m)]) since[size_t(m)] += run;
        HIPCHK(hipMemcpyAsync(rho.data(), sc.rho, Kb * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(act_now.data(), sc.active, Kb * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(sys_now.data(), sc.sys_active, K * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        bool any = false;
        for (int m = 0; m < K; ++m) {
            mask[size_t(m)] = 0;
            if (conv[size_t(m)]) continue;
            bool upd = it >= maxit || since[size_t(m)] >= inner_maxit;
            if (mixed) {
                for (int j = 0; j < b; ++j) {
                    const size_t q = size_t(m) * b + j;
                    if (act[q] && !(rho[q] > inner_tol * inner_tol * rho_last[q])) upd = true;  // NaN too
                }
            } else {
                upd = upd || !sys_now[size_t(m)];  // the recursion retired every column
            }
            if (upd) {
                mask[size_t(m)] = 1;
                any = true;
            }
        }
        if (!mixed) {
            // keep the host's view of the column flags in step with the recursion's
            for (size_t q = 0; q < Kb; ++q) act[q] = act_now[q];
            for (int m = 0; m < K; ++m) sysact[size_t(m)] = sys_now[size_t(m)];
        }
        if (any && (rc = refresh())) return rc;
        done = std::all_of(conv.begin(), conv.end(), [](int32_t c) { return c != 0; });
    }
    HIPCHK(hipMemcpyAsync(its.data(), iters_d, K * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (stats)
        for (int m = 0; m < K; ++m) {
            sell_cg_stats st;
            st.iterations = its[size_t(m)];
            st.refinements = refine[size_t(m)] > 0 ? refine[size_t(m)] - 1 : 0;
            st.relres = relres[size_t(m)];
            st.converged = conv[size_t(m)];
            stats[m] = st;
        }
    (void)Bview;
    return SELL_OK;
}

}  // extern "C"
