// blockops.cpp -- C ABI of the tall-skinny block-vector kernels (tsm.hip).
#include "internal.h"

namespace sellcs {
int launch_tsmttsm(const double *V, int64_t ldv, const double *W, int64_t ldw, int64_t n, int m, int k, double alpha,
                   double beta, double *X, int64_t ldx, int kahan, double *partials, int64_t max_partials,
                   hipStream_t s);
int launch_tsmm(const double *V, int64_t ldv, const double *X, int64_t ldx, int m, int k, int64_t n, double alpha,
                double beta, double *W, int64_t ldw, hipStream_t s);
int launch_tsmm_inplace(double *V, int64_t ldv, const double *X, int64_t ldx, int m, int64_t n, double alpha,
                        double beta, hipStream_t s);
}  // namespace sellcs

using namespace sellcs;

namespace {

int check_tall(const sell_bv *v) {
    if (!v) return SELL_ERR_ARG;
    if (v->dt != SELL_F64) return SELL_ERR_DTYPE;
    if (v->lay != SELL_ROW_MAJOR) return SELL_ERR_UNSUPPORTED;
    if (v->ncols < 1 || v->ncols > 64) return SELL_ERR_UNSUPPORTED;
    if (!v->ptr && v->nrows > 0) return SELL_ERR_ARG;
    return SELL_OK;
}

}  // namespace

extern "C" {

int sell_tsmttsm(const sell_bv *V, const sell_bv *W, double alpha, double beta, double *X, int64_t ldx, int kahan,
                 void *stream) {
    int rc;
    if ((rc = check_tall(V)) || (rc = check_tall(W))) return rc;
    if (V->nrows != W->nrows) return SELL_ERR_SHAPE;
    if (!X || ldx < W->ncols) return SELL_ERR_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace *ws = nullptr;
    if ((rc = get_workspace(s, &ws))) return rc;
    return launch_tsmttsm(static_cast<const double *>(V->ptr), V->ld, static_cast<const double *>(W->ptr), W->ld,
                          V->nrows, V->ncols, W->ncols, alpha, beta, X, ldx, kahan ? 1 : 0, ws->partials,
                          int64_t(kMaxTiles) * 3 * kMaxSliceCols, s);
}

int sell_tsmm(const sell_bv *V, const double *X, int64_t ldx, double alpha, double beta, sell_bv *W, void *stream) {
    int rc;
    if ((rc = check_tall(V)) || (rc = check_tall(W))) return rc;
    if (V->nrows != W->nrows) return SELL_ERR_SHAPE;
    if (!X || ldx < W->ncols) return SELL_ERR_ARG;
    if (V->ptr == W->ptr && V->nrows > 0) return SELL_ERR_ARG;
    return launch_tsmm(static_cast<const double *>(V->ptr), V->ld, X, ldx, V->ncols, W->ncols, V->nrows, alpha, beta,
                       static_cast<double *>(W->ptr), W->ld, static_cast<hipStream_t>(stream));
}

int sell_tsmm_inplace(sell_bv *V, const double *X, int64_t ldx, double alpha, double beta, void *stream) {
    int rc;
    if ((rc = check_tall(V))) return rc;
    if (!X || ldx < V->ncols) return SELL_ERR_ARG;
    return launch_tsmm_inplace(static_cast<double *>(V->ptr), V->ld, X, ldx, V->ncols, V->nrows, alpha, beta,
                               static_cast<hipStream_t>(stream));
}

}  // extern "C"
