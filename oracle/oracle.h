/*
 * oracle.h -- plain CPU FP64 reference for the augmented sparse matrix (multiple)
 * vector product and the SELL-C-sigma layout of the GHOST paper.
 *
 * TEST INFRASTRUCTURE ONLY. This is the oracle the HIP library is checked against.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg load it;
 * the library never includes, links or calls anything here, and nothing here
 * includes the library. Every routine is the plain definition of what it computes,
 * written on CSR input in IEEE double precision, in the simplest order.
 *
 * Conventions shared by all routines:
 *   CSR: rowptr int64[nrows+1], col int32[nnz], val double[nnz]; entries of a row are
 *        used in stored order; duplicated (row, col) pairs count as separate entries.
 *   Block vectors are row-major: element (i, j) of X lives at X[i * ldx + j].
 *   Return value: 0 on success, -1 on a bad argument.
 */
#ifndef SELL_ORACLE_H
#define SELL_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Augmentation switches of the fused product (paper Sec. 5.3); each one is
 * independent of the others. */
#define ORC_SHIFT 1u        /* subtract gamma * x (one scalar gamma)           */
#define ORC_VSHIFT 2u       /* subtract gamma_j * x_j (one gamma per column)    */
#define ORC_SCALE 4u        /* multiply by alpha                                */
#define ORC_AXPBY 8u        /* add beta * y_old                                 */
#define ORC_DOT_YY 16u      /* <y, y> per column of the final y                 */
#define ORC_DOT_XY 32u      /* <x, y> per column                                */
#define ORC_DOT_XX 64u      /* <x, x> per column                                */
#define ORC_CHAIN 128u      /* z = delta * z + eta * y  (final y)               */

/* Y = A X  (Sec. 5.1/5.2): Y[i,j] = sum_p val[p] * X[col[p], j], p over row i in order. */
int orc_spmmv(int64_t nrows, const int64_t *rowptr, const int32_t *col, const double *val,
              int64_t b, const double *X, int64_t ldx, double *Y, int64_t ldy);

/* Augmented product (Sec. 5.3):  y = alpha * (A - gamma I) x + beta * y,
 * optional dots of the final y, optional chained z = delta z + eta y.
 * alpha is 1 unless ORC_SCALE; gamma is 0 unless ORC_SHIFT/ORC_VSHIFT;
 * beta is 0 unless ORC_AXPBY, and y is not read when beta is 0; z is not read when
 * delta is 0.  dot (3*b doubles, may be NULL when no dot flag is set) receives
 * [<y,y>_0..b-1 | <x,y>_0..b-1 | <x,x>_0..b-1]; entries of unrequested dots are left
 * untouched.  Shifts and x-dots need a square matrix (x and y share row indices). */
int orc_spmmv_aug(int64_t nrows, int64_t ncols, const int64_t *rowptr, const int32_t *col,
                  const double *val, int64_t b, const double *X, int64_t ldx, double *Y,
                  int64_t ldy, double *Z, int64_t ldz, unsigned flags, double alpha, double beta,
                  double gamma, const double *gamma_v, double delta, double eta, double *dot);

/* <a, b> = sum_i a[i*inca] * b[i*incb], Neumaier-compensated, in index order. */
double orc_dot(int64_t n, const double *a, int64_t inca, const double *b, int64_t incb);

/* Y = A^T X: Y (ncols x b) is zeroed, then Y[col[p], j] += val[p] * X[i, j] row by row. */
int orc_spmmv_T(int64_t nrows, int64_t ncols, const int64_t *rowptr, const int32_t *col,
                const double *val, int64_t b, const double *X, int64_t ldx, double *Y,
                int64_t ldy);

/* SELL-C-sigma chunk structure (Sec. 5.1), by brute force:
 *   rows are sorted by descending length, ties in original order, inside windows of
 *   sigma consecutive rows (the last window may be short); the sorted rows are cut into
 *   chunks of C; a chunk's length is its longest row; chunk c starts at
 *   cs[c] = sum_{c' < c} C * cl[c'].
 * perm: int32[nch * C], slot -> original row, -1 for the empty slots past nrows.
 * cl: int32[nch]; cs: int64[nch + 1]; nch = ceil(nrows / C). */
int orc_sell_layout(int64_t nrows, const int64_t *rowptr, int64_t C, int64_t sigma,
                    int32_t *perm, int32_t *cl, int64_t *cs);

/* SELL-C-sigma arrays from CSR and a layout from orc_sell_layout: entry k of the row in
 * slot r of chunk c sits at cs[c] + k*C + r ("column-wise" inside the chunk); slots
 * past a row's end hold val 0 and col -1. */
int orc_sell_fill(int64_t nrows, const int64_t *rowptr, const int32_t *col, const double *val,
                  int64_t C, const int32_t *perm, const int32_t *cl, const int64_t *cs,
                  int32_t *scol, double *sval);

/* Round to the nearest bfloat16 (8 significant bits, binary32 exponent range) or binary32
 * value, ties to even, directly from the double; results returned as doubles. */
int orc_round_bf16(int64_t n, const double *in, double *out);
int orc_round_f32(int64_t n, const double *in, double *out);

/* Conjugate gradients (Hestenes-Stiefel) in FP64 for one right-hand side, x updated in
 * place from its initial value. Stops when ||r_k|| <= tol * ||b|| on the recursively
 * updated residual or after maxit iterations. *iters gets the iteration count. */
int orc_cg(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
           const double *bvec, double *x, double tol, int64_t maxit, int64_t *iters);

/* Iterative refinement around a CG in a lower inner precision (float vectors and products
 * when single != 0; double dots and scalars), values val_low for the inner products, FP64
 * residuals b - A x outside; restarts the inner CG from d = 0 at every refinement and stops
 * it when its residual has dropped to inner_rtol of the current true residual (or after
 * inner_maxit steps). *outer: refinements, *inner: total inner steps, *relres: final
 * ||b - A x|| / ||b||. */
int orc_cg_refine(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                  const double *val_low, const double *bvec, double *x, double tol, double inner_rtol,
                  int64_t inner_maxit, int64_t maxouter, int single, int64_t *outer, int64_t *inner,
                  double *relres);

/* Chebyshev recurrence of the kernel polynomial method for A~ = (A - c I) / s:
 *   v0 = x, v1 = A~ v0, v_{m+1} = 2 A~ v_m - v_{m-1};
 * mu[m] = <v0, v_m> for m = 0..M (the textbook moments, no doubling trick);
 * vlast (n doubles, may be NULL) receives v_M. */
int orc_chebyshev(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                  const double *x, int64_t M, double s, double c, double *mu, double *vlast);

/* Block Chebyshev application Y = T_N(A~) X for A~ = (A - c I) / s (three-term recurrence,
 * X and Y row-major n x b), and the gradient of a scalar loss L(Y) given G = dL/dY:
 *   dX   (n x b)  = dL/dX
 *   dval (nnz)    = dL/dval[p] for every stored entry p of A (CSR order),
 * by the adjoint (reverse-mode) recurrence with every v_m stored. N >= 1. */
int orc_cheb_apply(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, int64_t b,
                   const double *X, int64_t N, double s, double c, double *Y);
int orc_cheb_grad(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, int64_t b,
                  const double *X, int64_t N, double s, double c, const double *G, double *dX,
                  double *dval);

/* Chebyshev filter Z = sum_{m=0}^{N} coef[m] T_m(A~) X (X, Z row-major n x b), N >= 0. */
int orc_cheb_filter(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, int64_t b,
                    const double *X, int64_t N, const double *coef, double s, double c, double *Z);

/* dval[p] = sum_j G[row(p), j] * X[col[p], j]: the gradient of <G, A X> with respect to the
 * stored values (CSR order). */
int orc_pattern_outer(int64_t nrows, const int64_t *rowptr, const int32_t *col, int64_t b,
                      const double *G, const double *X, double *dval);

/* Tall-skinny block-vector kernels (Sec. 5.2); V: n x m, W: n x k row-major, X: m x k
 * row-major (small).
 *   tsmttsm:      X = alpha V^T W + beta X   (sums over the n rows in row order; kahan != 0:
 *                 Neumaier-compensated sums; X not read when beta == 0)
 *   tsmm:         W = alpha V X + beta W     (W not read when beta == 0)
 *   tsmm_inplace: V = alpha V X + beta V     (X is m x m; every row uses only its own old row) */
int orc_tsmttsm(int64_t n, int64_t m, int64_t k, double alpha, const double *V, const double *W, double beta,
                double *X, int kahan);
int orc_tsmm(int64_t n, int64_t m, int64_t k, double alpha, const double *V, const double *X, double beta,
             double *W);
int orc_tsmm_inplace(int64_t n, int64_t m, double alpha, double *V, const double *X, double beta);

/* Threads the oracle's parallel loops use (OpenMP), for reporting. */
int orc_num_threads(void);

/* Sets the threads of the oracle's later parallel loops (n >= 1; other values are ignored). */
void orc_set_num_threads(int n);

/* STREAM triad a = b + s c over n doubles (host bandwidth probe for the baseline's report,
 * not part of the product). Returns 0, or -1 for a negative n or a missing array. */
int orc_triad(int64_t n, double *a, const double *b, const double *c, double s);

#ifdef __cplusplus
}
#endif
#endif
