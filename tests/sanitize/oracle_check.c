/* The C oracle's routines run on random inputs under AddressSanitizer and
 * UndefinedBehaviorSanitizer: every routine with several block widths, every augmentation
 * flag combination, empty rows, long rows and duplicate columns, and CG on a 1D Laplacian.
 * Only memory safety and defined behaviour are checked here (values are pinned by the Python
 * tests). Exit status 0 when every call returns 0. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "oracle.h"

static uint64_t st = 1507;
static uint64_t rnd(void) {
    st += 0x9E3779B97F4A7C15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static double urand(void) { return (double)(rnd() >> 11) / 9007199254740992.0 * 2.0 - 1.0; }

static double *vec(int64_t n) {
    double *v = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) v[i] = urand();
    return v;
}

#define CHECK(call)                                        \
    do {                                                   \
        if ((call) != 0) {                                 \
            fprintf(stderr, "FAIL %s line %d\n", #call, __LINE__); \
            return 1;                                      \
        }                                                  \
    } while (0)

int main(void) {
    int calls = 0;
    for (int rep = 0; rep < 12; ++rep) {
        const int64_t n = (int64_t)(rnd() % 400);
        int64_t *rp = malloc(sizeof(int64_t) * (size_t)(n + 1));
        rp[0] = 0;
        int64_t cap = 16, nnz = 0;
        int32_t *col = malloc(sizeof(int32_t) * (size_t)cap);
        double *val = malloc(sizeof(double) * (size_t)cap);
        for (int64_t i = 0; i < n; ++i) {
            int64_t len = (int64_t)(rnd() % 9);
            if (rnd() % 40 == 0) len = (int64_t)(rnd() % 200);
            for (int64_t k = 0; k < len; ++k) {
                if (nnz == cap) {
                    cap *= 2;
                    col = realloc(col, sizeof(int32_t) * (size_t)cap);
                    val = realloc(val, sizeof(double) * (size_t)cap);
                }
                col[nnz] = (int32_t)(rnd() % (uint64_t)n);
                val[nnz] = urand();
                ++nnz;
            }
            rp[i + 1] = nnz;
        }
        const int64_t widths[] = {1, 3, 8};
        for (int w = 0; w < 3; ++w) {
            const int64_t b = widths[w];
            double *X = vec(n * b), *Y = vec(n * b), *Z = vec(n * b), *gv = vec(b), dot[3 * 8];
            CHECK(orc_spmmv(n, rp, col, val, b, X, b, Y, b));
            for (unsigned fl = 0; fl < 256; fl += 7) {
                CHECK(orc_spmmv_aug(n, n, rp, col, val, b, X, b, Y, b, Z, b, fl, 0.5, -1.0, 0.1, gv, 0.3, 2.0, dot));
                ++calls;
            }
            CHECK(orc_spmmv_T(n, n, rp, col, val, b, X, b, Y, b));
            CHECK(orc_cheb_apply(n, rp, col, val, b, X, 5, 4.0, 0.1, Y));
            double *G = vec(n * b), *dX = vec(n * b), *dval = vec(nnz), coef[6] = {1, 0.5, 0.25, 0.1, 0.05, 0.01};
            CHECK(orc_cheb_grad(n, rp, col, val, b, X, 5, 4.0, 0.1, G, dX, dval));
            CHECK(orc_cheb_filter(n, rp, col, val, b, X, 5, coef, 4.0, 0.1, Z));
            CHECK(orc_pattern_outer(n, rp, col, b, G, X, dval));
            double *Xs = vec(b * b);
            CHECK(orc_tsmttsm(n, b, b, 1.0, X, Y, 0.5, Xs, 1));
            CHECK(orc_tsmm(n, b, b, 1.0, X, Xs, 0.5, Y));
            CHECK(orc_tsmm_inplace(n, b, 1.0, X, Xs, 0.5));
            calls += 9;
            free(X); free(Y); free(Z); free(gv); free(G); free(dX); free(dval); free(Xs);
        }
        const int64_t Cs[] = {1, 8, 32};
        for (int c = 0; c < 3; ++c) {
            const int64_t C = Cs[c], nch = (n + C - 1) / C;
            int32_t *perm = malloc(sizeof(int32_t) * (size_t)(nch * C + 1));
            int32_t *cl = malloc(sizeof(int32_t) * (size_t)(nch + 1));
            int64_t *cs = malloc(sizeof(int64_t) * (size_t)(nch + 1));
            CHECK(orc_sell_layout(n, rp, C, n > 0 ? n : 1, perm, cl, cs));
            int32_t *scol = malloc(sizeof(int32_t) * (size_t)(cs[nch] + 1));
            double *sval = malloc(sizeof(double) * (size_t)(cs[nch] + 1));
            CHECK(orc_sell_fill(n, rp, col, val, C, perm, cl, cs, scol, sval));
            calls += 2;
            free(perm); free(cl); free(cs); free(scol); free(sval);
        }
        double *r1 = vec(nnz), *r2 = vec(nnz), *mu = vec(21), *vl = vec(n), *x0 = vec(n);
        CHECK(orc_round_bf16(nnz, val, r1));
        CHECK(orc_round_f32(nnz, val, r2));
        CHECK(orc_chebyshev(n, rp, col, val, x0, 10, 8.0, 0.0, mu, vl));
        calls += 3;
        free(r1); free(r2); free(mu); free(vl); free(x0); free(rp); free(col); free(val);
    }
    /* CG on the 1D Dirichlet Laplacian (SPD) */
    const int64_t n = 200;
    int64_t *rp = malloc(sizeof(int64_t) * (n + 1));
    int32_t *col = malloc(sizeof(int32_t) * 3 * n);
    double *val = malloc(sizeof(double) * 3 * n);
    int64_t p = 0;
    rp[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (i > 0) { col[p] = (int32_t)(i - 1); val[p++] = -1.0; }
        col[p] = (int32_t)i; val[p++] = 2.0;
        if (i < n - 1) { col[p] = (int32_t)(i + 1); val[p++] = -1.0; }
        rp[i + 1] = p;
    }
    double *bv = vec(n), *x = calloc((size_t)n, sizeof(double));
    int64_t it = 0;
    CHECK(orc_cg(n, rp, col, val, bv, x, 1e-10, 1000, &it));
    free(rp); free(col); free(val); free(bv); free(x);
    printf("oracle: %d calls ok\n", calls + 1);
    return 0;
}
