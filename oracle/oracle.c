/*
 * oracle.c -- plain CPU FP64 reference for the GHOST paper's augmented sparse matrix
 * (multiple) vector product (Sec. 5.3), its block-vector form (Sec. 5.2) and the
 * SELL-C-sigma layout (Sec. 5.1).
 *
 * TEST INFRASTRUCTURE ONLY: the checker, not the product. It is built with
 * -ffp-contract=off so every multiply and add rounds separately, exactly as written.
 * SELL-C-sigma is a lossless re-layout of the matrix, so the product it must reach is
 * the plain CSR product; that plain definition is what is written here.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Host memory bandwidth probe for reporting beside the baseline (McCalpin's STREAM triad):
 * a = b + s c over n doubles, in the same static split of the loop as the oracle's products. */
int orc_triad(int64_t n, double *a, const double *b, const double *c, double s) {
    if (n < 0 || (n > 0 && (!a || !b || !c))) return -1;
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) a[i] = b[i] + s * c[i];
    return 0;
}

/* ---------------------------------------------------------------------------------
 * Sparse matrix times block vector (Sec. 5.1, 5.2): Y = A X, one row at a time, the
 * row's entries summed in stored order starting from +0.
 */
int orc_spmmv(int64_t nrows, const int64_t *rowptr, const int32_t *col, const double *val,
              int64_t b, const double *X, int64_t ldx, double *Y, int64_t ldy) {
    if (nrows < 0 || b < 1 || ldx < b || ldy < b) return -1;
    if (nrows == 0) return 0;
    if (!rowptr || !Y) return -1;
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < nrows; ++i) {
        for (int64_t j = 0; j < b; ++j) {
            double s = 0.0;
            for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
                s = s + val[p] * X[(int64_t)col[p] * ldx + j];
            Y[i * ldy + j] = s;
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------------------
 * Compensated dot product (Neumaier's improvement of Kahan summation; the paper adds a
 * Kahan-summed reduction for long inner products in Sec. 5.2).
 */
double orc_dot(int64_t n, const double *a, int64_t inca, const double *b, int64_t incb) {
    double s = 0.0, comp = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double term = a[i * inca] * b[i * incb];
        double t = s + term;
        if (fabs(s) >= fabs(term))
            comp += (s - t) + term;
        else
            comp += (term - t) + s;
        s = t;
    }
    return s + comp;
}

/* ---------------------------------------------------------------------------------
 * Augmented product (Sec. 5.3):  y = alpha (A - gamma I) x + beta y, then dots of the
 * final y and the chained z = delta z + eta y.
 */
int orc_spmmv_aug(int64_t nrows, int64_t ncols, const int64_t *rowptr, const int32_t *col,
                  const double *val, int64_t b, const double *X, int64_t ldx, double *Y,
                  int64_t ldy, double *Z, int64_t ldz, unsigned flags, double alpha, double beta,
                  double gamma, const double *gamma_v, double delta, double eta, double *dot) {
    const unsigned need_square = ORC_SHIFT | ORC_VSHIFT | ORC_DOT_XY | ORC_DOT_XX;
    if (nrows < 0 || ncols < 0 || b < 1 || ldx < b || ldy < b) return -1;
    if ((flags & need_square) && nrows != ncols) return -1;
    if ((flags & ORC_VSHIFT) && !gamma_v) return -1;
    if ((flags & ORC_CHAIN) && (!Z || ldz < b)) return -1;
    if ((flags & (ORC_DOT_YY | ORC_DOT_XY | ORC_DOT_XX)) && !dot) return -1;

    double *s = (double *)malloc(sizeof(double) * (size_t)(nrows > 0 ? nrows : 1) * (size_t)b);
    if (!s) return -1;
    /* step 1: s = A x */
    int rc = orc_spmmv(nrows, rowptr, col, val, b, X, ldx, s, b);
    if (rc) {
        free(s);
        return rc;
    }
    const double a = (flags & ORC_SCALE) ? alpha : 1.0;
    const double bt = (flags & ORC_AXPBY) ? beta : 0.0;
    /* step 2: y = a * (s - g_j x) + bt * y_old   (y_old only read when bt != 0) */
    for (int64_t i = 0; i < nrows; ++i) {
        for (int64_t j = 0; j < b; ++j) {
            double g = 0.0;
            if (flags & ORC_VSHIFT)
                g = gamma_v[j];
            else if (flags & ORC_SHIFT)
                g = gamma;
            double t = s[i * b + j];
            if (flags & (ORC_SHIFT | ORC_VSHIFT)) t = t - g * X[i * ldx + j];
            double y = a * t;
            if (bt != 0.0) y = y + bt * Y[i * ldy + j];
            Y[i * ldy + j] = y;
        }
    }
    free(s);
    /* step 3: dots of the final y */
    for (int64_t j = 0; j < b; ++j) {
        if (flags & ORC_DOT_YY) dot[j] = orc_dot(nrows, Y + j, ldy, Y + j, ldy);
        if (flags & ORC_DOT_XY) dot[b + j] = orc_dot(nrows, X + j, ldx, Y + j, ldy);
        if (flags & ORC_DOT_XX) dot[2 * b + j] = orc_dot(nrows, X + j, ldx, X + j, ldx);
    }
    /* step 4: z = delta z + eta y   (z only read when delta != 0) */
    if (flags & ORC_CHAIN) {
        for (int64_t i = 0; i < nrows; ++i)
            for (int64_t j = 0; j < b; ++j) {
                double z = eta * Y[i * ldy + j];
                if (delta != 0.0) z = delta * Z[i * ldz + j] + z;
                Z[i * ldz + j] = z;
            }
    }
    return 0;
}

/* ---------------------------------------------------------------------------------
 * Transposed product Y = A^T X by scattering each row's contribution.
 */
int orc_spmmv_T(int64_t nrows, int64_t ncols, const int64_t *rowptr, const int32_t *col,
                const double *val, int64_t b, const double *X, int64_t ldx, double *Y,
                int64_t ldy) {
    if (nrows < 0 || ncols < 0 || b < 1 || ldx < b || ldy < b) return -1;
    for (int64_t c = 0; c < ncols; ++c)
        for (int64_t j = 0; j < b; ++j) Y[c * ldy + j] = 0.0;
    for (int64_t i = 0; i < nrows; ++i)
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
            for (int64_t j = 0; j < b; ++j)
                Y[(int64_t)col[p] * ldy + j] = Y[(int64_t)col[p] * ldy + j] + val[p] * X[i * ldx + j];
    return 0;
}

/* ---------------------------------------------------------------------------------
 * SELL-C-sigma layout (Sec. 5.1) by brute force.
 */
static const int64_t *g_len_for_sort; /* row lengths for the comparator below */

static int by_length_desc_then_index(const void *pa, const void *pb) {
    int32_t ra = *(const int32_t *)pa, rb = *(const int32_t *)pb;
    int64_t la = g_len_for_sort[ra], lb = g_len_for_sort[rb];
    if (la != lb) return la > lb ? -1 : 1; /* longer rows first */
    return ra < rb ? -1 : (ra > rb ? 1 : 0); /* equal lengths keep their original order */
}

int orc_sell_layout(int64_t nrows, const int64_t *rowptr, int64_t C, int64_t sigma,
                    int32_t *perm, int32_t *cl, int64_t *cs) {
    if (nrows < 0 || C < 1 || sigma < 1) return -1;
    int64_t nch = (nrows + C - 1) / C;
    int64_t *len = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nrows > 0 ? nrows : 1));
    if (!len) return -1;
    for (int64_t i = 0; i < nrows; ++i) len[i] = rowptr[i + 1] - rowptr[i];
    for (int64_t s = 0; s < nch * C; ++s) perm[s] = s < nrows ? (int32_t)s : -1;
    g_len_for_sort = len;
    for (int64_t w = 0; w < nrows; w += sigma) {
        int64_t we = w + sigma < nrows ? w + sigma : nrows;
        qsort(perm + w, (size_t)(we - w), sizeof(int32_t), by_length_desc_then_index);
    }
    g_len_for_sort = NULL;
    cs[0] = 0;
    for (int64_t c = 0; c < nch; ++c) {
        int64_t m = 0;
        for (int64_t r = 0; r < C; ++r) {
            int32_t row = perm[c * C + r];
            if (row >= 0 && len[row] > m) m = len[row];
        }
        cl[c] = (int32_t)m;
        cs[c + 1] = cs[c] + C * m;
    }
    free(len);
    return 0;
}

int orc_sell_fill(int64_t nrows, const int64_t *rowptr, const int32_t *col, const double *val,
                  int64_t C, const int32_t *perm, const int32_t *cl, const int64_t *cs,
                  int32_t *scol, double *sval) {
    if (nrows < 0 || C < 1) return -1;
    int64_t nch = (nrows + C - 1) / C;
    for (int64_t c = 0; c < nch; ++c)
        for (int64_t r = 0; r < C; ++r) {
            int32_t row = perm[c * C + r];
            int64_t len = row >= 0 ? rowptr[row + 1] - rowptr[row] : 0;
            for (int64_t k = 0; k < cl[c]; ++k) {
                int64_t at = cs[c] + k * C + r;
                if (k < len) {
                    scol[at] = col[rowptr[row] + k];
                    sval[at] = val[rowptr[row] + k];
                } else {
                    scol[at] = -1;
                    sval[at] = 0.0;
                }
            }
        }
    return 0;
}

/* ---------------------------------------------------------------------------------
 * Rounding to bfloat16 / binary32, nearest with ties to even, taken straight from the
 * definition: the representable neighbours of v are the multiples of the quantum
 * q = 2^(e - p) for v = f * 2^e with 0.5 <= |f| < 1 and p significant bits (clamped at
 * the subnormal quantum), so v rounds to q * nearbyint(v / q) in the default rounding
 * mode (which breaks ties to the even multiple). Dividing by a power of two is exact.
 */
static double round_to_format(double v, int p, int emin_sub, double maxfinite) {
    if (!isfinite(v) || v == 0.0) return v;
    int e;
    frexp(v, &e);
    int qe = e - p;
    if (qe < emin_sub) qe = emin_sub;
    double q = ldexp(1.0, qe);
    double r = nearbyint(v / q) * q;
    if (fabs(r) > maxfinite) return v > 0 ? INFINITY : -INFINITY;
    return r;
}

int orc_round_bf16(int64_t n, const double *in, double *out) {
    /* bfloat16: 8 significant bits, smallest subnormal 2^-133, largest finite
     * (2 - 2^-7) * 2^127 */
    const double maxf = ldexp(2.0 - ldexp(1.0, -7), 127);
    for (int64_t i = 0; i < n; ++i) out[i] = round_to_format(in[i], 8, -133, maxf);
    return 0;
}

int orc_round_f32(int64_t n, const double *in, double *out) {
    /* binary32: 24 significant bits, smallest subnormal 2^-149 */
    const double maxf = ldexp(2.0 - ldexp(1.0, -23), 127);
    for (int64_t i = 0; i < n; ++i) out[i] = round_to_format(in[i], 24, -149, maxf);
    return 0;
}

/* ---------------------------------------------------------------------------------
 * Conjugate gradients, textbook Hestenes-Stiefel form, FP64.
 */
int orc_cg(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
           const double *bvec, double *x, double tol, int64_t maxit, int64_t *iters) {
    if (n < 0 || maxit < 0) return -1;
    size_t sz = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *r = (double *)malloc(sz), *p = (double *)malloc(sz), *q = (double *)malloc(sz);
    if (!r || !p || !q) {
        free(r);
        free(p);
        free(q);
        return -1;
    }
    orc_spmmv(n, rowptr, col, val, 1, x, 1, q, 1);
    for (int64_t i = 0; i < n; ++i) {
        r[i] = bvec[i] - q[i];
        p[i] = r[i];
    }
    double bnorm = sqrt(orc_dot(n, bvec, 1, bvec, 1));
    double rr = orc_dot(n, r, 1, r, 1);
    int64_t it = 0;
    while (it < maxit && sqrt(rr) > tol * bnorm) {
        orc_spmmv(n, rowptr, col, val, 1, p, 1, q, 1);
        double alpha = rr / orc_dot(n, p, 1, q, 1);
        for (int64_t i = 0; i < n; ++i) {
            x[i] = x[i] + alpha * p[i];
            r[i] = r[i] - alpha * q[i];
        }
        double rr_new = orc_dot(n, r, 1, r, 1);
        double beta = rr_new / rr;
        for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        rr = rr_new;
        ++it;
    }
    if (iters) *iters = it;
    free(r);
    free(p);
    free(q);
    return 0;
}

/* ---------------------------------------------------------------------------------
 * Iterative refinement with a low-precision inner CG: the reference for the iteration counts
 * of the refined solver (CG is only named by the paper; refinement is the textbook scheme).
 *   r = b - A x                          (FP64 values, FP64 arithmetic)
 *   while ||r|| > tol ||b|| and fewer than maxouter refinements:
 *       d = 0; CG on A_low d = r from d = 0 until its recursive residual has dropped to
 *           inner_rtol ||r|| or after inner_maxit steps; A_low holds val_low (the values in
 *           the inner storage precision, given as doubles); with single != 0 the vectors and
 *           the products are float (each product term and sum rounded to float), the dots and
 *           the scalars double; with single == 0 everything is double
 *       x = x + d;  r = b - A x          (FP64)
 * *outer gets the refinements, *inner the CG steps over all of them, *relres the final
 * ||b - A x|| / ||b||.
 */
static void orc_spmv_f32(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                         const float *x, float *y) {
    for (int64_t i = 0; i < n; ++i) {
        float acc = 0.0f;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            const float prod = (float)val[p] * x[col[p]];
            acc = acc + prod;
        }
        y[i] = acc;
    }
}

static double orc_dot_f32(int64_t n, const float *a, const float *b) {
    double s = 0.0, c = 0.0; /* Neumaier, as orc_dot */
    for (int64_t i = 0; i < n; ++i) {
        const double t = (double)a[i] * (double)b[i];
        const double u = s + t;
        if (fabs(s) >= fabs(t))
            c += (s - u) + t;
        else
            c += (t - u) + s;
        s = u;
    }
    return s + c;
}

int orc_cg_refine(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                  const double *val_low, const double *bvec, double *x, double tol, double inner_rtol,
                  int64_t inner_maxit, int64_t maxouter, int single, int64_t *outer, int64_t *inner,
                  double *relres) {
    if (n < 0 || inner_maxit < 0 || maxouter < 0) return -1;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    double *r = (double *)malloc(sizeof(double) * nn), *t = (double *)malloc(sizeof(double) * nn);
    double *dd = (double *)malloc(sizeof(double) * nn), *pd = (double *)malloc(sizeof(double) * nn);
    double *qd = (double *)malloc(sizeof(double) * nn), *rd = (double *)malloc(sizeof(double) * nn);
    float *df = (float *)malloc(sizeof(float) * nn), *pf = (float *)malloc(sizeof(float) * nn);
    float *qf = (float *)malloc(sizeof(float) * nn), *rf = (float *)malloc(sizeof(float) * nn);
    int rc = 0;
    if (!r || !t || !dd || !pd || !qd || !rd || !df || !pf || !qf || !rf) {
        rc = -1;
        goto done;
    }
    const double bnorm = sqrt(orc_dot(n, bvec, 1, bvec, 1));
    int64_t nout = 0, nin = 0;
    orc_spmmv(n, rowptr, col, val, 1, x, 1, t, 1);
    for (int64_t i = 0; i < n; ++i) r[i] = bvec[i] - t[i];
    double rnorm = sqrt(orc_dot(n, r, 1, r, 1));
    while (rnorm > tol * bnorm && nout < maxouter) {
        const double stop = inner_rtol * rnorm;
        int64_t it = 0;
        if (single) {
            for (int64_t i = 0; i < n; ++i) {
                df[i] = 0.0f;
                rf[i] = (float)r[i];
                pf[i] = rf[i];
            }
            double rr = orc_dot_f32(n, rf, rf);
            while (it < inner_maxit && sqrt(rr) > stop) {
                orc_spmv_f32(n, rowptr, col, val_low, pf, qf);
                const double alpha = rr / orc_dot_f32(n, pf, qf);
                for (int64_t i = 0; i < n; ++i) {
                    df[i] = (float)((double)df[i] + alpha * (double)pf[i]);
                    rf[i] = (float)((double)rf[i] - alpha * (double)qf[i]);
                }
                const double rr_new = orc_dot_f32(n, rf, rf);
                const double beta = rr_new / rr;
                for (int64_t i = 0; i < n; ++i) pf[i] = (float)((double)rf[i] + beta * (double)pf[i]);
                rr = rr_new;
                ++it;
            }
            for (int64_t i = 0; i < n; ++i) x[i] = x[i] + (double)df[i];
        } else {
            for (int64_t i = 0; i < n; ++i) {
                dd[i] = 0.0;
                rd[i] = r[i];
                pd[i] = rd[i];
            }
            double rr = orc_dot(n, rd, 1, rd, 1);
            while (it < inner_maxit && sqrt(rr) > stop) {
                orc_spmmv(n, rowptr, col, val_low, 1, pd, 1, qd, 1);
                const double alpha = rr / orc_dot(n, pd, 1, qd, 1);
                for (int64_t i = 0; i < n; ++i) {
                    dd[i] = dd[i] + alpha * pd[i];
                    rd[i] = rd[i] - alpha * qd[i];
                }
                const double rr_new = orc_dot(n, rd, 1, rd, 1);
                const double beta = rr_new / rr;
                for (int64_t i = 0; i < n; ++i) pd[i] = rd[i] + beta * pd[i];
                rr = rr_new;
                ++it;
            }
            for (int64_t i = 0; i < n; ++i) x[i] = x[i] + dd[i];
        }
        nin += it;
        ++nout;
        orc_spmmv(n, rowptr, col, val, 1, x, 1, t, 1);
        for (int64_t i = 0; i < n; ++i) r[i] = bvec[i] - t[i];
        rnorm = sqrt(orc_dot(n, r, 1, r, 1));
        if (it == 0) break; /* no progress possible (inner_rtol >= 1 or inner_maxit == 0) */
    }
    if (outer) *outer = nout;
    if (inner) *inner = nin;
    if (relres) *relres = bnorm > 0.0 ? rnorm / bnorm : rnorm;
done:
    free(r);
    free(t);
    free(dd);
    free(pd);
    free(qd);
    free(rd);
    free(df);
    free(pf);
    free(qf);
    free(rf);
    return rc;
}

/* ---------------------------------------------------------------------------------
 * Chebyshev recurrence of the kernel polynomial method, direct moments.
 */
int orc_chebyshev(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                  const double *x, int64_t M, double s, double c, double *mu, double *vlast) {
    if (n < 0 || M < 0 || s == 0.0) return -1;
    size_t sz = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *vprev = (double *)malloc(sz), *vcur = (double *)malloc(sz), *t = (double *)malloc(sz);
    if (!vprev || !vcur || !t) {
        free(vprev);
        free(vcur);
        free(t);
        return -1;
    }
    memcpy(vcur, x, sizeof(double) * (size_t)n);
    mu[0] = orc_dot(n, x, 1, vcur, 1);
    for (int64_t m = 1; m <= M; ++m) {
        orc_spmmv(n, rowptr, col, val, 1, vcur, 1, t, 1);
        for (int64_t i = 0; i < n; ++i) {
            double at = (t[i] - c * vcur[i]) / s; /* A~ v_{m-1} */
            double next = (m == 1) ? at : 2.0 * at - vprev[i];
            vprev[i] = vcur[i];
            t[i] = next;
        }
        double *sw = vcur;
        vcur = t;
        t = sw;
        mu[m] = orc_dot(n, x, 1, vcur, 1);
    }
    if (vlast) memcpy(vlast, vcur, sizeof(double) * (size_t)n);
    free(vprev);
    free(vcur);
    free(t);
    return 0;
}

/* ---------------------------------------------------------------------------------
 * Chebyshev application and its gradient (reverse mode written out by hand).
 * Forward: v_0 = X, v_1 = A~ v_0, v_{m+1} = 2 A~ v_m - v_{m-1}, Y = v_N, A~ = (A - cI)/s.
 * Adjoint: with w_m = dL/dv_m, w_N = G; walking m = N-1 .. 1 over v_{m+1} = 2 A~ v_m - v_{m-1}:
 *   w_m += 2 A~^T w_{m+1},  w_{m-1} -= w_{m+1},  dval += (2/s) outer(w_{m+1}, v_m);
 * then for v_1 = A~ v_0:  w_0 += A~^T w_1,  dval += (1/s) outer(w_1, v_0); dX = w_0.
 */
static void atilde(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, int64_t b,
                   const double *V, double s, double c, double *out) {
    orc_spmmv(n, rowptr, col, val, b, V, b, out, b);
    for (int64_t e = 0; e < n * b; ++e) out[e] = (out[e] - c * V[e]) / s;
}

static void atilde_T(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, int64_t b,
                     const double *W, double s, double c, double *out) {
    orc_spmmv_T(n, n, rowptr, col, val, b, W, b, out, b);
    for (int64_t e = 0; e < n * b; ++e) out[e] = (out[e] - c * W[e]) / s;
}

int orc_pattern_outer(int64_t nrows, const int64_t *rowptr, const int32_t *col, int64_t b,
                      const double *G, const double *X, double *dval) {
    if (nrows < 0 || b < 1) return -1;
    for (int64_t i = 0; i < nrows; ++i)
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            double acc = 0.0;
            for (int64_t j = 0; j < b; ++j) acc = acc + G[i * b + j] * X[(int64_t)col[p] * b + j];
            dval[p] = acc;
        }
    return 0;
}

int orc_cheb_apply(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, int64_t b,
                   const double *X, int64_t N, double s, double c, double *Y) {
    if (n < 0 || b < 1 || N < 1 || s == 0.0) return -1;
    size_t sz = sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)b;
    double *prev = (double *)malloc(sz), *cur = (double *)malloc(sz), *nxt = (double *)malloc(sz);
    if (!prev || !cur || !nxt) {
        free(prev);
        free(cur);
        free(nxt);
        return -1;
    }
    memcpy(prev, X, sizeof(double) * (size_t)(n * b));
    atilde(n, rowptr, col, val, b, prev, s, c, cur);
    for (int64_t m = 1; m < N; ++m) {
        atilde(n, rowptr, col, val, b, cur, s, c, nxt);
        for (int64_t e = 0; e < n * b; ++e) nxt[e] = 2.0 * nxt[e] - prev[e];
        double *t = prev;
        prev = cur;
        cur = nxt;
        nxt = t;
    }
    memcpy(Y, cur, sizeof(double) * (size_t)(n * b));
    free(prev);
    free(cur);
    free(nxt);
    return 0;
}

/* Chebyshev filter Z = sum_{m=0}^{N} coef[m] T_m(A~) X: the recurrence as in orc_cheb_apply,
 * with every v_m added into Z, scaled by its coefficient, right after it is formed. N >= 0. */
int orc_cheb_filter(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, int64_t b,
                    const double *X, int64_t N, const double *coef, double s, double c, double *Z) {
    if (n < 0 || b < 1 || N < 0 || s == 0.0 || !coef) return -1;
    const size_t ne = (size_t)n * (size_t)b;
    size_t sz = sizeof(double) * (ne > 0 ? ne : 1);
    double *prev = (double *)malloc(sz), *cur = (double *)malloc(sz), *nxt = (double *)malloc(sz);
    if (!prev || !cur || !nxt) {
        free(prev);
        free(cur);
        free(nxt);
        return -1;
    }
    for (size_t e = 0; e < ne; ++e) {
        prev[e] = X[e];
        Z[e] = coef[0] * X[e];
    }
    if (N >= 1) {
        atilde(n, rowptr, col, val, b, prev, s, c, cur);
        for (size_t e = 0; e < ne; ++e) Z[e] += coef[1] * cur[e];
    }
    for (int64_t m = 1; m < N; ++m) {
        atilde(n, rowptr, col, val, b, cur, s, c, nxt);
        for (size_t e = 0; e < ne; ++e) {
            nxt[e] = 2.0 * nxt[e] - prev[e];
            Z[e] += coef[m + 1] * nxt[e];
        }
        double *t = prev;
        prev = cur;
        cur = nxt;
        nxt = t;
    }
    free(prev);
    free(cur);
    free(nxt);
    return 0;
}

int orc_cheb_grad(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, int64_t b,
                  const double *X, int64_t N, double s, double c, const double *G, double *dX,
                  double *dval) {
    if (n < 0 || b < 1 || N < 1 || s == 0.0) return -1;
    const int64_t nb = n * b;
    const int64_t nnz = rowptr[n];
    double *V = (double *)malloc(sizeof(double) * (size_t)(N + 1) * (size_t)(nb > 0 ? nb : 1));
    double *W = (double *)calloc((size_t)(N + 1) * (size_t)(nb > 0 ? nb : 1), sizeof(double));
    double *t = (double *)malloc(sizeof(double) * (size_t)(nb > 0 ? nb : 1));
    double *dv = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    if (!V || !W || !t || !dv) {
        free(V);
        free(W);
        free(t);
        free(dv);
        return -1;
    }
    /* forward, keeping every v_m */
    memcpy(V, X, sizeof(double) * (size_t)nb);
    atilde(n, rowptr, col, val, b, V, s, c, V + nb);
    for (int64_t m = 1; m < N; ++m) {
        atilde(n, rowptr, col, val, b, V + m * nb, s, c, V + (m + 1) * nb);
        for (int64_t e = 0; e < nb; ++e) V[(m + 1) * nb + e] = 2.0 * V[(m + 1) * nb + e] - V[(m - 1) * nb + e];
    }
    /* reverse */
    for (int64_t p = 0; p < nnz; ++p) dval[p] = 0.0;
    memcpy(W + N * nb, G, sizeof(double) * (size_t)nb);
    for (int64_t m = N - 1; m >= 1; --m) {
        const double *wn = W + (m + 1) * nb;
        atilde_T(n, rowptr, col, val, b, wn, s, c, t);
        for (int64_t e = 0; e < nb; ++e) {
            W[m * nb + e] += 2.0 * t[e];
            W[(m - 1) * nb + e] -= wn[e];
        }
        orc_pattern_outer(n, rowptr, col, b, wn, V + m * nb, dv);
        for (int64_t p = 0; p < nnz; ++p) dval[p] += (2.0 / s) * dv[p];
    }
    atilde_T(n, rowptr, col, val, b, W + nb, s, c, t);
    for (int64_t e = 0; e < nb; ++e) W[e] += t[e];
    orc_pattern_outer(n, rowptr, col, b, W + nb, V, dv);
    for (int64_t p = 0; p < nnz; ++p) dval[p] += (1.0 / s) * dv[p];
    memcpy(dX, W, sizeof(double) * (size_t)nb);
    free(V);
    free(W);
    free(t);
    free(dv);
    return 0;
}

/* ---------------------------------------------------------------------------------
 * Tall-skinny block-vector kernels (Sec. 5.2), plain loops.
 */
int orc_tsmttsm(int64_t n, int64_t m, int64_t k, double alpha, const double *V, const double *W, double beta,
                double *X, int kahan) {
    if (n < 0 || m < 1 || k < 1) return -1;
    for (int64_t l = 0; l < m; ++l)
        for (int64_t j = 0; j < k; ++j) {
            double s = 0.0, comp = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                const double term = V[i * m + l] * W[i * k + j];
                if (kahan) {
                    const double t = s + term;
                    if (fabs(s) >= fabs(term))
                        comp += (s - t) + term;
                    else
                        comp += (term - t) + s;
                    s = t;
                } else {
                    s = s + term;
                }
            }
            const double v = alpha * (s + comp);
            X[l * k + j] = beta != 0.0 ? v + beta * X[l * k + j] : v;
        }
    return 0;
}

int orc_tsmm(int64_t n, int64_t m, int64_t k, double alpha, const double *V, const double *X, double beta,
             double *W) {
    if (n < 0 || m < 1 || k < 1) return -1;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < k; ++j) {
            double s = 0.0;
            for (int64_t l = 0; l < m; ++l) s = s + V[i * m + l] * X[l * k + j];
            const double v = alpha * s;
            W[i * k + j] = beta != 0.0 ? v + beta * W[i * k + j] : v;
        }
    return 0;
}

int orc_tsmm_inplace(int64_t n, int64_t m, double alpha, double *V, const double *X, double beta) {
    if (n < 0 || m < 1) return -1;
    double *row = (double *)malloc(sizeof(double) * (size_t)m);
    if (!row) return -1;
    for (int64_t i = 0; i < n; ++i) {
        memcpy(row, V + i * m, sizeof(double) * (size_t)m);
        for (int64_t j = 0; j < m; ++j) {
            double s = 0.0;
            for (int64_t l = 0; l < m; ++l) s = s + row[l] * X[l * m + j];
            const double v = alpha * s;
            V[i * m + j] = beta != 0.0 ? v + beta * row[j] : v;
        }
    }
    free(row);
    return 0;
}
