// solvers.cpp -- conjugate-gradient drivers (placeholder until the CG kernels land).
#include "internal.h"

extern "C" {

int sell_cg(const sell_mat *, const sell_bv *, sell_bv *, double, int64_t, sell_cg_stats *, void *) {
    return SELL_ERR_UNSUPPORTED;
}

int sell_cg_mixed(const sell_mat *, const sell_mat *, const sell_bv *, sell_bv *, double, int64_t, double,
                  int64_t, sell_cg_stats *, void *) {
    return SELL_ERR_UNSUPPORTED;
}

}  // extern "C"
