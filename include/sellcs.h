/*
 * sellcs.h -- C ABI of libsellcs: SELL-C-sigma sparse matrix times (block) vector,
 * plain and augmented, for one AMD Instinct MI355X (gfx950).
 *
 * What is computed follows the GHOST paper (Kreutzer et al., "GHOST: Building blocks for
 * high performance sparse linear algebra on heterogeneous systems"):
 *   - the SELL-C-sigma storage format (Sec. 5.1): rows cut into chunks of C, each chunk
 *     padded with trailing zeros to its longest row and stored column by column, rows
 *     sorted by length inside windows of sigma rows;
 *   - block vectors (Sec. 3.2, 5.2): tall, skinny dense matrices, preferably row-major
 *     ("interleaved"), usable as views of memory the caller owns;
 *   - the augmented product (Sec. 5.3):  y = alpha (A - gamma I) x + beta y, fused with
 *     the dot products <y,y>, <x,y>, <x,x> and the chained z = delta z + eta y, each
 *     augmentation switched on separately.
 *
 * General rules for every entry point:
 *   - Return value: SELL_OK (0) or a negative SELL_ERR_* code; sell_strerror() names it.
 *     No C++ exception crosses this interface. Arguments are checked before any GPU work
 *     is issued; a call that fails a check has no effect.
 *   - "stream" is a hipStream_t passed as void* (NULL = the default stream). Compute calls
 *     are asynchronous on that stream: they enqueue kernels and return. Results (including
 *     dot products, which land in device memory) are valid once the stream has reached
 *     that point.
 *   - All device memory passed in must belong to the current HIP device.
 *   - Indices: local row and column indices are 32-bit (nrows, ncols < 2^31); offsets into
 *     the stored arrays are 64-bit, so a matrix may store more than 2^31 entries
 *     (Sec. 5.1 discusses 32-bit local indices).
 *   - Environment overrides of launch shapes, read once per process, for tuning
 *     experiments (every row is computed the same way under all of them; dot products may
 *     differ in the last bits, from another split of the partial sums):
 *       SELLCS_VPT=1|2|4           columns per lane of the fixed-width kernels (default up to 4)
 *       SELLCS_BLOCKS_PER_CU=n     workgroups per compute unit of a resident grid (1..64;
 *                                  default from the kernel's occupancy)
 *       SELLCS_TILES=n             fine tiles of a matrix built afterwards (1..4096; default 4096)
 *       SELLCS_BATCH_WAVES=n       grid of a batched product in waves of resident workgroups
 *                                  (1..32; default 16)
 *       SELLCS_XCD_MAP=0           plain workgroup-to-tile order instead of contiguous tile
 *                                  ranges per XCD
 *     The per-matrix setters (sell_set_launch, sell_set_waves, sell_set_batch, sell_set_slice)
 *     take precedence where they apply.
 *   - Diagnostics on stderr (the performance-warning and information lines of Sec. 4.1):
 *       SELLCS_LOG=0|1|2           0 or unset: none; 1: a "[sellcs] PERFWARNING" line, once per
 *                                  process and cause, when a product runs its slower
 *                                  run-time-width kernel (a block width other than 1, 2, 4,
 *                                  8, 16, 32, or block vectors that are not row-major with
 *                                  aligned rows) or the atomic transpose; 2: also a
 *                                  "[sellcs] INFO" line for each build (shape, stored
 *                                  entries, chunks, tiles, batch length, grid) and each
 *                                  autotuning result
 */
#ifndef SELLCS_H
#define SELLCS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sell_mat sell_mat; /* opaque SELL-C-sigma matrix            */
typedef struct sell_bv sell_bv;   /* opaque block vector (owner or view)   */

/* Element types. Matrix values may be F64, F32 or BF16; block vectors F64, F32 or BF16
 * (BF16 block vectors are storage only: sell_bv_copy converts them, the products do not
 * take them). */
typedef enum { SELL_F64 = 0, SELL_F32 = 1, SELL_BF16 = 2 } sell_dtype;

/* Block-vector storage (Sec. 3.2): row-major = interleaved, element (i, j) at
 * ptr[i * ld + j]; column-major: element (i, j) at ptr[j * ld + i]. */
typedef enum { SELL_ROW_MAJOR = 0, SELL_COL_MAJOR = 1 } sell_layout;

enum {
    SELL_OK = 0,
    SELL_ERR_ARG = -1,         /* null pointer, bad size or bad parameter          */
    SELL_ERR_SHAPE = -2,       /* operand dimensions do not fit together           */
    SELL_ERR_DTYPE = -3,       /* element-type combination not offered             */
    SELL_ERR_UNSUPPORTED = -4, /* valid request that this library does not do      */
    SELL_ERR_OOM = -5,         /* device or host allocation failed                  */
    SELL_ERR_HIP = -6,         /* a HIP runtime call failed                         */
    SELL_ERR_STATE = -7        /* object not in a usable state (e.g. host-only)     */
};

/* ------------------------------------------------------------------------------------ */
/* Library                                                                              */

/* Static text for an error code (never NULL). */
const char *sell_strerror(int code);

/* Library version as 10000*major + 100*minor + patch. */
int sell_version(void);

/* Test hooks for the error paths (not for production use). sell_debug_fail_alloc(k): the k-th
 * device or pinned host allocation the library makes from now on fails as out of memory
 * (k >= 1; 0 clears; the hook is process-wide). sell_debug_live_allocs: the number of device
 * and pinned host allocations the library holds (its workspaces and the objects alive), so that
 * a test can check that a failed call left nothing behind. Errors: SELL_ERR_ARG for k < 0 or a
 * NULL count. */
int sell_debug_fail_alloc(int64_t k);
int sell_debug_live_allocs(int64_t *count);

/* ------------------------------------------------------------------------------------ */
/* Sparse matrix (Sec. 3.1, 5.1)                                                        */

/* Build a SELL-C-sigma matrix on the current device from host CSR arrays (Sec. 5.1
 * describes construction from raw CRS data).
 *   rowptr: int64[nrows + 1], rowptr[0] = 0, non-decreasing; col: int32[nnz] with
 *   0 <= col < ncols; val: double[nnz]. Entries of a row keep their order; duplicated
 *   (row, col) pairs stay separate entries. The host arrays are only read, and are not
 *   referenced after the call returns.
 *   C >= 1 (chunk height), 1 <= sigma (sorting window; sigma > nrows acts as nrows).
 *   Rows are sorted by descending length inside each window of sigma rows, ties keeping
 *   their original order; sigma = 1 keeps the original order.
 *   vdt: storage type of the values; F64 values are converted to F32 or BF16 by
 *   rounding to nearest, ties to even, directly from the double.
 * On success *A owns device memory; release it with sell_destroy. The call returns after
 * the upload has finished (it synchronises "stream").
 * Errors: SELL_ERR_ARG (null pointers, C < 1, sigma < 1, rowptr not monotone or
 * rowptr[0] != 0, a column outside [0, ncols), nrows or ncols >= 2^31),
 * SELL_ERR_DTYPE, SELL_ERR_OOM, SELL_ERR_HIP. */
int sell_build(sell_mat **A, int64_t nrows, int64_t ncols, const int64_t *rowptr,
               const int32_t *col, const double *val, int32_t C, int64_t sigma,
               sell_dtype vdt, void *stream);

/* Same as sell_build for a CSR matrix already in DEVICE memory (rowptr, col, val are device
 * pointers on the current device): every step of the construction runs on the GPU (row
 * lengths, the stable sort inside sigma windows, chunk lengths and starts, the column-major
 * fill with padding and value conversion), and the result is identical to sell_build's entry
 * for entry. The small per-chunk arrays, the permutation and the row pointers are also kept in
 * host memory, as for sell_build. The input arrays are only read. Invalid CSR input (row
 * pointers not starting at 0 or decreasing, column indices out of range) gives SELL_ERR_ARG.
 * Synchronous (returns when the matrix is ready). */
int sell_build_device(sell_mat **A, int64_t nrows, int64_t ncols, const int64_t *rowptr,
                      const int32_t *col, const double *val, int32_t C, int64_t sigma,
                      sell_dtype vdt, void *stream);

/* Same as sell_build but keeps the SELL arrays in host memory only and touches no GPU.
 * The result serves sell_info, sell_export_csr, sell_export_sell and sell_destroy; the
 * compute calls reject it with SELL_ERR_STATE. */
int sell_build_host(sell_mat **A, int64_t nrows, int64_t ncols, const int64_t *rowptr,
                    const int32_t *col, const double *val, int32_t C, int64_t sigma,
                    sell_dtype vdt);

/* Replace the values of a matrix with the same sparsity pattern (Sec. 5.1: later
 * constructions with an unchanged pattern only update values).
 *   val: double[nnz] in the CSR order given at build time, in host memory
 *   (sell_update_values) or device memory (sell_update_values_device). Converted to the
 *   matrix's storage type. Asynchronous on "stream" for the device variant; the host
 *   variant returns after the copy. */
int sell_update_values(sell_mat *A, const double *val, void *stream);
int sell_update_values_device(sell_mat *A, const double *val, void *stream);

/* Copy the matrix back out as CSR into caller-owned host arrays (rowptr int64[nrows+1],
 * col int32[nnz], val double[nnz]). For an F64 matrix this reproduces the build input
 * bit for bit; F32/BF16 values come back as the doubles they represent. */
int sell_export_csr(const sell_mat *A, int64_t *rowptr, int32_t *col, double *val);

/* Copy the raw SELL-C-sigma arrays into caller-owned host arrays (any may be NULL):
 *   perm int32[nchunks*C] (slot -> original row, -1 for slots past the last row),
 *   cl int32[nchunks] (chunk lengths), cs int64[nchunks+1] (chunk starts),
 *   col int32[stored] and val double[stored] (entry k of slot r of chunk c at
 *   cs[c] + k*C + r; padding has col = -1 and val = 0). */
int sell_export_sell(const sell_mat *A, int32_t *perm, int32_t *cl, int64_t *cs,
                     int32_t *col, double *val);

typedef struct {
    int64_t nrows, ncols;
    int64_t nnz;           /* true nonzeros                                      */
    int64_t stored;        /* stored entries including padding                  */
    int64_t nchunks;       /* ceil(nrows / C)                                    */
    int64_t sigma;
    int32_t C;
    int32_t vdtype;        /* sell_dtype of the values                           */
    int32_t on_device;     /* 1 for sell_build results, 0 for sell_build_host    */
    int32_t device;        /* HIP device id (-1 if host-only)                    */
    int32_t ntiles;        /* work partitions of one product launch              */
    int32_t has_perm;      /* 0 when the row order is unchanged (sigma = 1)      */
    int64_t matrix_bytes;  /* bytes of all device arrays of the matrix           */
    int32_t batch;         /* index batch length of the products (5, 7 or 8; see
                              sell_set_batch)                                     */
    int32_t batch_wide;    /* the same for the kernels that gather 32 bytes per
                              lane (FP64, 4 columns per lane: b >= 4)             */
} sell_info_t;

int sell_info(const sell_mat *A, sell_info_t *out);

/* Free a matrix (device and host memory). NULL is a no-op. Must not race with work
 * still queued on a stream that uses A. */
int sell_destroy(sell_mat *A);

/* ------------------------------------------------------------------------------------ */
/* Block vectors (Sec. 3.2, 5.2)                                                        */

/* Create an nrows x ncols block vector of type dt and layout lay on the current device.
 *   data == NULL: the library allocates (ld is then ignored and set to ncols for
 *   row-major, nrows for column-major) and owns the memory; the contents are zeroed.
 *   data != NULL: a view of caller-owned device memory (Sec. 3.2 "views of raw data",
 *   e.g. a torch tensor), never freed by the library; ld >= ncols (row-major) or
 *   ld >= nrows (column-major).
 * nrows >= 0, 1 <= ncols. */
int sell_bv_create(sell_bv **X, int64_t nrows, int32_t ncols, sell_dtype dt, sell_layout lay,
                   void *data, int64_t ld);

/* Free an owned block vector, or forget a view. NULL is a no-op. */
int sell_bv_destroy(sell_bv *X);

/* Pointer, leading dimension and shape of a block vector (any out-pointer may be NULL). */
int sell_bv_data(const sell_bv *X, void **data, int64_t *ld, int64_t *nrows, int32_t *ncols,
                 int32_t *dtype, int32_t *layout);

/* dst = src elementwise, converting layout (row-/column-major, Sec. 3.2) and element type
 * (F64 <-> F32 <-> BF16, narrowing by round to nearest, ties to even). Shapes must agree;
 * dst and src must not overlap unless they are the same object with the same type and
 * layout (then nothing is done). Asynchronous on stream. */
int sell_bv_copy(sell_bv *dst, const sell_bv *src, void *stream);

/* ------------------------------------------------------------------------------------ */
/* Products (Sec. 5.2, 5.3)                                                             */

/* Y = A X (Sec. 5.1, 5.2). X: ncols x b, Y: nrows x b, both row- or column-major.
 * Types: F64 matrix with F64 vectors (FP64 arithmetic); F32 or BF16 matrix with F32
 * vectors (FP32 accumulation). Y must not overlap X. Deterministic: repeated calls give
 * identical bits. */
int sell_spmmv(const sell_mat *A, const sell_bv *X, sell_bv *Y, void *stream);

/* Augmentation switches (Sec. 5.3); combine with |. Each one is independent. */
#define SELL_SPMV_SHIFT 0x01u  /* subtract gamma * x, one gamma for all columns      */
#define SELL_SPMV_VSHIFT 0x02u /* subtract gamma_v[j] * x_j, one per column           */
#define SELL_SPMV_SCALE 0x04u  /* multiply by alpha                                   */
#define SELL_SPMV_AXPBY 0x08u  /* add beta * y (y is not read when beta == 0)        */
#define SELL_SPMV_DOT_YY 0x10u /* <y, y> per column of the final y                    */
#define SELL_SPMV_DOT_XY 0x20u /* <x, y> per column                                   */
#define SELL_SPMV_DOT_XX 0x40u /* <x, x> per column                                   */
#define SELL_SPMV_CHAIN 0x80u  /* z = delta z + eta y (z not read when delta == 0)    */
#define SELL_SPMV_DOTS (SELL_SPMV_DOT_YY | SELL_SPMV_DOT_XY | SELL_SPMV_DOT_XX)

typedef struct {
    uint32_t flags;
    double alpha;          /* used with SELL_SPMV_SCALE, else 1                       */
    double beta;           /* used with SELL_SPMV_AXPBY, else 0                       */
    double gamma;          /* used with SELL_SPMV_SHIFT                               */
    const double *gamma_v; /* HOST array of b shifts, with SELL_SPMV_VSHIFT; read
                              before the call returns                                 */
    double delta, eta;     /* used with SELL_SPMV_CHAIN                               */
    double *dot;           /* DEVICE array of 3*b doubles receiving
                              [<y,y>_0..b-1 | <x,y>_0..b-1 | <x,x>_0..b-1];
                              entries of dots not requested are left untouched        */
} sell_spmv_opts;

/* Defaults: alpha = 1, beta = 0, gamma = 0, delta = 0, eta = 1, no flags. */
#define SELL_SPMV_OPTS_INIT {0u, 1.0, 0.0, 0.0, (const double *)0, 0.0, 1.0, (double *)0}

/* Augmented product (Sec. 5.3):
 *   y <- alpha (A x - gamma_j x) + beta y ;  dots of the final y ;  z <- delta z + eta y.
 * All arithmetic of the epilogue is FP64; the dots are accumulated in FP64 for every
 * type and are computed from the stored y. Shifts and x-dots need a square A. Z (same
 * shape and type as Y) is required with SELL_SPMV_CHAIN, else ignored (may be NULL).
 * opts == NULL means the defaults. Deterministic, dots included (fixed reduction order,
 * no floating-point atomics). Concurrent calls with dots on different streams are safe;
 * calls with dots on one stream are ordered by the stream. */
int sell_spmmv_aug(const sell_mat *A, const sell_bv *X, sell_bv *Y, sell_bv *Z,
                   const sell_spmv_opts *opts, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): sell_spmmv_aug with the same arguments, kernels and
 * results, bit for bit, but no allocation. sell_spmmv_aug keeps its dot partials in a workspace
 * that it allocates on its first call on each stream; this variant keeps them, with the
 * kernels' lane scratch, in a fixed array of 6,324,224 bytes per device (3 dots x 64 columns x
 * 4,096 workgroups of FP64 partials, plus 32 KiB), which each device holds until the process
 * ends. The first call on a device looks up the array's address (hipGetSymbolAddress); later
 * calls only launch kernels. Every call on a device shares the array: calls that overlap on one
 * device (other streams, other threads) race on it and must be ordered by the caller. Returns
 * SELL_ERR_UNSUPPORTED if a launch could need more partials than the array holds (a matrix with
 * more than 4,096 work tiles; the library never builds one), else the errors of sell_spmmv_aug. */
int sell_spmmv_aug_noalloc(const sell_mat *A, const sell_bv *X, sell_bv *Y, sell_bv *Z,
                           const sell_spmv_opts *opts, void *stream);

/* Y = A^T X. X: nrows x b, Y: ncols x b, row-major. deterministic = 1 (the recommended
 * choice and the Python binding's default) runs the forward kernel on a SELL-C-sigma copy of
 * A^T, which the first such call builds and keeps with A (a synchronous, allocating call that
 * holds a second copy of the matrix); later calls are bit-reproducible and on the 128^3 Anderson
 * matrix at b = 8 about 23x faster than the atomic form. deterministic = 0 scatters with
 * floating-point atomics, needs no copy, and may differ in the last bits from run to run. */
int sell_spmmv_T(const sell_mat *A, const sell_bv *X, sell_bv *Y, int deterministic,
                 void *stream);

/* ------------------------------------------------------------------------------------ */
/* Solver drivers built from the products (Sec. 5.2 block BLAS-1 operations, Sec. 6)    */

/* Kernel polynomial method recurrence for A~ = (A - c I) / s on a block of starting
 * vectors: v_0 = V (nrows x b, F64 row-major, overwritten), v_1 = A~ v_0,
 * v_{m+1} = 2 A~ v_m - v_{m-1}, using M augmented products with fused dots.
 * mu (DEVICE, (2M + 1) * b doubles, column j's moments at mu[m * b + j]) receives the
 * Chebyshev moments mu_m = <v_0, T_m(A~) v_0> for m = 0..2M, from the doubling
 * identities mu_2m = 2 <v_m, v_m> - mu_0 and mu_2m+1 = 2 <v_m+1, v_m> - mu_1.
 * W is a work block vector of the same shape. On return V and W hold v_M and v_{M-1}
 * (which one holds which is reported in *last_in_w, may be NULL). M >= 1.
 * step_ms: NULL for an asynchronous call; else a HOST array of M floats that receives the
 * duration of each augmented product, timed with HIP events recorded on "stream" between
 * consecutive launches (created with hipEventDisableSystemFence: timing only, no cache
 * writeback and invalidation at each record; the call synchronises the stream before it
 * reads them and returns). */
int sell_kpm(const sell_mat *A, sell_bv *V, sell_bv *W, int64_t M, double s, double c,
             double *mu, int *last_in_w, float *step_ms, void *stream);

/* Density of states from block KPM moments (the kernel polynomial method that the fused
 * block product serves, Sec. 5.3; the reconstruction is the standard one): the b columns'
 * moments are summed and normalised, mu~_m = sum_j mu[m * b + j] / sum_j mu[j] (a stochastic
 * trace estimate when the columns are random vectors), damped with kernel (SELL_KPM_JACKSON:
 * g_m = ((N - m + 1) cos(pi m / (N + 1)) + sin(pi m / (N + 1)) cot(pi / (N + 1))) / (N + 1)
 * with N = nmom; SELL_KPM_NONE: g_m = 1), and summed as a Chebyshev series:
 *   rho[k] = (g_0 mu~_0 + 2 sum_{m=1}^{nmom-1} g_m mu~_m T_m(x)) / (pi sqrt(1 - x^2) s),
 *   x = (E[k] - c) / s,  rho[k] = 0 where |x| >= 1,
 * the density per unit energy of A when A~ = (A - c I) / s (the scaling of sell_kpm).
 * mu: DEVICE, nmom * b doubles in sell_kpm's layout (nmom = 2M + 1 there). E, rho: DEVICE,
 * K doubles each (may be NULL when K = 0). sum_j mu[j] must be nonzero (else rho is not
 * finite). Deterministic (fixed summation order). Asynchronous.
 * Errors: SELL_ERR_ARG for nmom < 1, b < 1, K < 0, another kernel, s not positive or not
 * finite, c not finite, or a NULL pointer that is needed. */
enum { SELL_KPM_NONE = 0, SELL_KPM_JACKSON = 1 };
int sell_kpm_dos(const double *mu, int64_t nmom, int32_t b, int32_t kernel, double s, double c,
                 const double *E, int64_t K, double *rho, void *stream);

typedef struct {
    int64_t iterations;       /* total inner (low-precision) or plain CG iterations  */
    int64_t refinements;      /* outer FP64 residual corrections (0 for plain CG)     */
    double relres;            /* max over columns of ||b - A x|| / ||b|| (FP64)       */
    int32_t converged;        /* 1 if relres <= tol                                   */
} sell_cg_stats;

/* Conjugate gradients for each column of B (A symmetric positive definite, F64 matrix,
 * F64 row-major vectors). X holds the initial guess and receives the solution. Stops
 * when every column has ||b - A x|| <= tol ||b|| (true FP64 residual, checked every few
 * iterations) or after maxit iterations. Synchronous (returns when done). An iteration is
 * one product q = A p with the fused <q, q> and <p, q>, and one vector pass r -= alpha q,
 * x += alpha p, p = r + beta p with beta = (alpha^2 <q, q> - rho) / rho, which equals
 * <r', r'> / rho in exact arithmetic (the single-reduction form of Rupp et al., ACM TOMS
 * 43(2), 2016); rho = <r, r> is summed directly and decides convergence. sell_cg_mixed and
 * sell_batch_cg iterate the same way. */
int sell_cg(const sell_mat *A, const sell_bv *B, sell_bv *X, double tol, int64_t maxit,
            sell_cg_stats *stats, void *stream);

/* Mixed-precision CG with FP64 iterative refinement by reliable updates: CG runs in FP32
 * vectors on the F32 or BF16 matrix Alo (same pattern as A64) and accumulates its correction
 * d in FP32. Whenever the FP32 residual has dropped by the factor inner_tol (0 < inner_tol < 1)
 * since the last update, or after inner_maxit iterations, d is added to x in FP64 and the
 * residual is replaced by the true r = b - A64 x computed in FP64 with the F64 matrix A64;
 * the search direction is kept. Stops at the same criterion as sell_cg (true FP64 residual
 * <= tol ||b|| per column) or after maxit iterations in total. Synchronous. */
int sell_cg_mixed(const sell_mat *A64, const sell_mat *Alo, const sell_bv *B, sell_bv *X,
                  double tol, int64_t maxit, double inner_tol, int64_t inner_maxit,
                  sell_cg_stats *stats, void *stream);

/* ------------------------------------------------------------------------------------ */
/* Derivatives with respect to the stored values (used by automatic differentiation)    */

/* dval[p] (+)= alpha * sum_j G[row(p), j] X[col(p), j] for every stored entry p, CSR order:
 * the gradient of <G, A X> with respect to the values of A (a pattern-restricted outer
 * product). G: nrows x b, X: ncols x b, row-major with ld = b, the matrix's vector type;
 * dval: DEVICE array of nnz doubles, overwritten (accumulate = 0) or added to (1).
 * Asynchronous. */
int sell_grad_values(const sell_mat *A, const sell_bv *G, const sell_bv *X, double alpha,
                     int accumulate, double *dval, void *stream);

/* Y = T_N(A~) X with A~ = (A - c I) / s, by the Chebyshev three-term recurrence
 * v_0 = X, v_1 = A~ v_0, v_m+1 = 2 A~ v_m - v_m-1 (each step one augmented product).
 * A square; X, Y: n x b row-major with ld = b, b <= 64, the matrix's vector type.
 * ckpt: NULL, or a DEVICE buffer of 2 * ceil(N / K) * n * b elements of the vector type
 * that receives the pairs (v_kK, v_kK+1) for the backward pass. N >= 1, K >= 1.
 * Asynchronous. */
int sell_cheb_forward(const sell_mat *A, const sell_bv *X, sell_bv *Y, int64_t N, double s,
                      double c, int64_t K, void *ckpt, void *stream);

/* Chebyshev filter Z = sum_{m=0}^{N} coef[m] T_m(A~) X with A~ = (A - c I) / s (polynomial
 * filters and expansions such as exp(t A~); Sec. 5.3's chained axpby): z = coef[0] x, then
 * every step of the recurrence is one augmented product that forms v_m+1 and, chained in the
 * same kernel, z = z + coef[m+1] v_m+1. A square; X, Z: n x b row-major with ld = b, b <= 64,
 * the matrix's vector type, Z != X. coef: HOST array of N + 1 doubles, N >= 0. Two work blocks
 * are allocated in stream order. Asynchronous. */
int sell_cheb_filter(const sell_mat *A, const sell_bv *X, sell_bv *Z, int64_t N, const double *coef,
                     double s, double c, void *stream);

/* Adjoint of sell_cheb_forward for a scalar loss L with G = dL/dY: dX = dL/dX and
 * dval = dL/dval (DEVICE, nnz doubles, CSR order), from the checkpoints of the forward call
 * with the same (N, s, c, K) and the same matrix values. Each segment of K steps is
 * recomputed from its checkpoint; A^T products use the SELL copy of A^T (built on the
 * first call, a synchronous allocating call). Asynchronous otherwise. */
int sell_cheb_backward(const sell_mat *A, const sell_bv *G, int64_t N, double s, double c,
                       int64_t K, const void *ckpt, sell_bv *dX, double *dval, void *stream);

/* ------------------------------------------------------------------------------------ */
/* Tall-skinny block-vector kernels (Sec. 5.2)                                          */
/* V: n x m, W: n x k block vectors (F64, row-major, 1 <= m, k <= 64); X: small m x k (or
 * m x m) DEVICE matrix, row-major with leading dimension ldx. Asynchronous. */

/* X = alpha V^T W + beta X (inner product of block vectors; X not read when beta == 0).
 * Deterministic FP64 reduction over the n rows; kahan != 0 uses compensated (Neumaier)
 * summation in every partial and in the final sum. */
int sell_tsmttsm(const sell_bv *V, const sell_bv *W, double alpha, double beta, double *X,
                 int64_t ldx, int kahan, void *stream);

/* W = alpha V X + beta W (W not read when beta == 0; W must not overlap V). */
int sell_tsmm(const sell_bv *V, const double *X, int64_t ldx, double alpha, double beta,
              sell_bv *W, void *stream);

/* V = alpha V X + beta V with X m x m: each row of V is read completely before it is
 * overwritten. */
int sell_tsmm_inplace(sell_bv *V, const double *X, int64_t ldx, double alpha, double beta,
                      void *stream);

/* ------------------------------------------------------------------------------------ */
/* Parameter choice                                                                     */
/*                                                                                      */
/* The paper chooses C from the hardware's vector width and sigma between padding and    */
/* right-hand-side locality (Sec. 5.1); the best values depend on the device and on the  */
/* matrix, so they are found here by timed trials on the device (micro-benchmarks, as    */
/* planned for device-dependent choices in Sec. 7.2).                                    */

/* Launch parameters of the product kernels for this matrix: columns per lane of the
 * fixed-width kernels (1, 2 or 4, at most the block width; 0 = default: 4 for b >= 4, else b)
 * and workgroups per compute unit (1..64, capped at the occupancy limit; 0 = the default:
 * one where a lane gathers 32 bytes per entry (FP64 vectors, 4 columns per lane), else the
 * occupancy limit).
 * Results do not depend on them (every row is computed the same way); dot products may
 * differ in the last bits (another split of the partial sums). */
int sell_set_launch(sell_mat *A, int32_t vpt, int32_t blocks_per_cu);

/* Grid of the product launches of A in waves of resident workgroups: waves in {0, 1, 2, 4, 8,
 * 16}; 0 restores the construction's choice: 16 waves when the chunk lengths spread widely
 * (coefficient of variation above 1/2), else one. Several waves let workgroups that finish early
 * take the next ones, which balances matrices whose tiles differ in speed (scattered gathers),
 * and keep the workgroups that run at the same time on neighbouring rows; the grid never
 * exceeds the matrix's fine tiles (at most 4096). Results per row are the same; dots may differ
 * in the last bits. */
int sell_set_waves(sell_mat *A, int32_t waves);

/* Processes blocks wider than `slice` columns (slice in {1, 2, 4, 8, 16, 32}; 0 = the whole
 * block in one launch) as consecutive launches over column slices of that width, when slice
 * divides the block width (else the default split). Applies to sell_spmmv and
 * sell_spmmv_aug (the dots of each slice land in their columns); the CG drivers ignore it.
 * Results per row are the same; dots may differ in the last bits. */
int sell_set_slice(sell_mat *A, int32_t slice);

/* Index batch length of the products of widths 1, 2, 4, 8, 16 and 32. A batched launch
 * (sell_batch_spmmv_aug, sell_batch_cg) uses the length its matrices share, and 8 when they
 * differ (the length is taken when the batch is created); the run-time-width kernel, the
 * packed mixed-width launch and the atomic transposed product keep 8. A lane loads
 * the column indices and values of `batch` consecutive entries of its row, then all their x
 * rows, then sums them; a chunk of L entries (Sec. 5.1: all rows of a chunk are padded to the
 * chunk's length) takes ceil(L / batch) such rounds, the last one re-reading its final entry
 * for the slots past L. batch in {5, 7, 8}: rows of 5 or 7 entries (2D and 3D stencils) then
 * waste no loads. 0 restores the construction's choice, which picks the length from the chunk
 * lengths: 5, 7 or 8, and 5 or 7 for the kernels whose lane gathers 32 bytes per entry (FP64
 * values and vectors at b >= 4), where 8-entry batches leave two waves per SIMD instead of
 * three. sell_info reports both (batch, batch_wide); a length set here applies to every
 * kernel. Results are the same bit for bit. */
int sell_set_batch(sell_mat *A, int32_t batch);

/* Gathering x through LDS (stage = 1). The rows of x form pages of 64 rows. For every work tile
 * the first product builds (once, synchronously: a kernel, then a wait on the stream) the
 * sorted list of the pages the tile's entries reference and 16-bit tile-local copies of its
 * column indices (page position, row in page; Sec. 4.1 compresses the column indices of the
 * remote part of a distributed matrix the same way). A workgroup then copies each tile's pages
 * into a cache of 144 KiB of LDS with contiguous loads, keeping the pages it already holds, and
 * gathers x from there; it reads the 2-byte indices instead of the 4-byte ones. Tiles with more
 * pages than the cache holds (at most 64) gather from global memory as before. Applies to the
 * single-matrix products at the fixed widths 1, 2, 4, 8, 16 and 32 with row-major x whose rows
 * are contiguous and 16-byte aligned; other calls ignore it.
 * tile_stride > 0 (staged launches): workgroup g takes the stage tiles g % S + S k of its share
 * of k (S = tile_stride) one after another instead of a contiguous range, where S divides the
 * number of stage tiles and of workgroups (else ignored): for a matrix whose far neighbours lie
 * S stage tiles away (the next plane of a 3D grid) consecutive tiles of a workgroup then share
 * most of their pages. A stage tile is one pass of the kernel (512 * columns per lane / b rows).
 * 0, 0 restores the defaults. y and z are the same bit for bit (every row sums the same entries
 * in the same order); the dots, summed over the rows in another grouping when a workgroup takes
 * its tiles one at a time, may differ in the last bits. Errors: SELL_ERR_ARG for stage outside
 * {0, 1} or a negative stride. */
int sell_set_stage(sell_mat *A, int32_t stage, int32_t tile_stride);

typedef struct {
    int32_t C;             /* chosen chunk height                                      */
    int64_t sigma;         /* chosen sorting window                                    */
    int32_t vpt;           /* chosen columns per lane (0 = default)                    */
    int32_t blocks_per_cu; /* chosen workgroups per compute unit (0 = sell_set_launch default) */
    double us;             /* time of one product with the choice (microseconds)       */
    double default_us;     /* the same for C = 32, sigma = 1 and the default launch    */
    int32_t trials;        /* configurations timed; 0 when answered from the cache     */
    int32_t slice;         /* chosen slice width for the block (0 = whole block)       */
    int32_t waves;         /* chosen grid in waves of resident workgroups (0 = one)    */
    int32_t batch;         /* chosen index batch length (0 = the construction's choice) */
} sell_tune_result;

#define SELL_TUNE_NO_CACHE 0x1u /* time the candidates even if the shape class is cached */

/* Times candidate formats of the CSR matrix (same arguments as sell_build) for products
 * with block width b (1..64) on the current device: C in {16, 32, 64} with sigma in
 * {1, 8 C, 256 C}, then columns per lane {1, 2, 4} and workgroups per CU {limit, 1, 2} for the
 * best pair, then grids of 2, 4 or 8 waves (sell_set_waves), then index batches of 5, 7 and 8
 * entries (sell_set_batch), then slices of 8, 16 or 32 columns that divide b (the b packing,
 * sell_set_slice);
 * a candidate replaces the best so far only when more than 3 % faster (the default,
 * C = 32, sigma = 1, is timed first). The trial product is the one a CG iteration issues (fused
 * <x, y>; plain for a rectangular matrix). Results are cached per process for the matrix's
 * shape class (value type, b, order of magnitude of the row count, mean row length,
 * row-length histogram over power-of-two bins). Synchronous; allocates and frees its own trial
 * matrices and vectors. */
int sell_autotune(int64_t nrows, int64_t ncols, const int64_t *rowptr, const int32_t *col,
                  const double *val, sell_dtype vdt, int32_t b, uint32_t flags,
                  sell_tune_result *out, void *stream);

/* ------------------------------------------------------------------------------------ */
/* Batches of independent matrices                                                      */
/*                                                                                      */
/* The paper distributes one matrix over heterogeneous devices by work weights which it  */
/* plans to derive from micro-benchmarks (Sec. 4.1 and the outlook, Sec. 7.2). On one    */
/* GPU the same idea spreads many small and uneven matrices over the compute units: one  */
/* launch processes every matrix of a batch, with the workgroups split by each matrix's   */
/* cost (stored entries plus rows) so that the busiest workgroup has the least work.      */

typedef struct sell_batch sell_batch;

/* Groups count >= 1 device matrices (same value type, current device) into a batch. The
 * batch refers to the matrices, which must outlive it; it allocates small device tables and
 * pinned staging memory. The block vectors of a batch hold the operands of its matrices one
 * after another: matrix m reads rows [c_m, c_m + ncols_m) of X and writes rows
 * [r_m, r_m + nrows_m) of Y, with r_m, c_m the sums of the earlier matrices' sizes. Launch
 * parameters set with sell_set_launch apply to the batch when all its matrices have the same
 * ones (read at creation); otherwise the defaults are used. */
int sell_batch_create(sell_mat *const *mats, int32_t count, sell_batch **out);
int sell_batch_destroy(sell_batch *B);
/* count of matrices and the total rows / columns of the stacked operands (each may be NULL) */
int sell_batch_info(const sell_batch *B, int32_t *count, int64_t *rows, int64_t *cols);

/* Y_m = alpha (A_m - gamma I) X_m + beta Y_m with dots and chain (opts exactly as for
 * sell_spmmv_aug, applied to every matrix) in one launch. X: total-columns x b, Y and Z:
 * total-rows x b, the batch's vector type, 1 <= b <= 64. opts->dot receives 3 b doubles per
 * matrix: matrix m's group q (yy = 0, xy = 1, xx = 2), column j at dot[(3 m + q) b + j].
 * SELL_ERR_UNSUPPORTED while block widths other than b are set (sell_batch_set_widths).
 * Calls on one batch must be ordered (one stream, or synchronised): the launch tables are
 * reused. Asynchronous. */
int sell_batch_spmmv_aug(sell_batch *B, const sell_bv *X, sell_bv *Y, sell_bv *Z,
                         const sell_spmv_opts *opts, void *stream);

/* Block widths of the batch's matrices, for batches whose systems have different numbers of
 * vectors (block widths 1..64 in one launch): widths is a HOST array of count entries, each in
 * [1, 64], or NULL to clear them. The widths define the packed operand layout of
 * sell_batch_spmmv_aug_packed. While widths other than b are set, sell_batch_spmmv_aug with
 * operands of width b returns SELL_ERR_UNSUPPORTED, and so does sell_batch_cg (both need one
 * width for all). Synchronous (waits for the device). Errors: SELL_ERR_ARG (NULL batch, width
 * out of range), SELL_ERR_STATE (another device is current). */
int sell_batch_set_widths(sell_batch *B, const int32_t *widths);

/* Sizes of the packed operands for the widths set (0 when none are set), each may be NULL:
 * elements of X (sum of ncols_m w_m), of Y and Z (sum of nrows_m w_m), and doubles of the dots
 * (3 sum of w_m). */
int sell_batch_packed_sizes(const sell_batch *B, int64_t *x_elems, int64_t *y_elems, int64_t *dots);

/* The product of sell_batch_spmmv_aug over packed operands of per-matrix widths, in one launch:
 * matrix m's X_m (ncols_m x w_m, row-major, leading dimension w_m) starts at element
 * sum_{k<m} ncols_k w_k of X, and its Y_m and Z_m (nrows_m x w_m) at element
 * sum_{k<m} nrows_k w_k of Y and Z. X, Y, Z: DEVICE, the batch's vector type (F64 for F64
 * values, else F32), aligned to the element size. opts as for sell_spmmv_aug, applied to every
 * matrix (gamma_v: at least max w_m entries, matrix m uses the first w_m); opts->dot receives
 * matrix m's dots packed at dot + 3 sum_{k<m} w_k, as [yy (w_m) | xy (w_m) | xx (w_m)].
 * Every workgroup runs the kernel body compiled for its matrix's width (run-time width for
 * widths outside 1, 2, 4, 8, 16, 32 or rows not aligned for 16-byte accesses); the workgroups
 * are split by each matrix's bytes at its own width. Asynchronous; calls on one batch must be
 * ordered. Errors: SELL_ERR_STATE (no widths set, or another device is current),
 * SELL_ERR_ARG (NULL or misaligned operand that is needed, X == Y, bad flags or missing
 * gamma_v / dot), SELL_ERR_SHAPE (shifts or x-dots with a non-square matrix). */
int sell_batch_spmmv_aug_packed(sell_batch *B, const void *X, void *Y, void *Z, const sell_spmv_opts *opts,
                                void *stream);

#define SELL_BATCH_GRAPH 0x1u /* capture the iterations in a HIP graph and replay it */

/* Conjugate gradients for every system m of a batch (A_m symmetric positive definite) and
 * every column of its right-hand sides: B and X are total-rows x b, F64, row-major with
 * ld = b, 1 <= b <= 64; X holds the initial guesses and receives the solutions. A64: batch
 * of F64 matrices. Alo: NULL for FP64 CG, else a batch of the same matrices with F32 or
 * BF16 values, for FP32 iterations refined in FP64 by reliable updates per system (the
 * scheme of sell_cg_mixed, with inner_tol and inner_maxit per system). A system stops when
 * every column has ||b - A x|| <= tol ||b|| (true FP64 residual); maxit bounds the
 * iterations of the batch. All systems advance together, a converged one is skipped by
 * every kernel. flags: 0 or SELL_BATCH_GRAPH. stats: NULL or a HOST array of count
 * entries (per system: its iterations, refinements, final relres, converged). Synchronous.
 * A NULL stream makes the call use a stream of its own (the legacy default stream cannot
 * be captured), ordered after earlier work on the default stream. */
int sell_batch_cg(sell_batch *A64, sell_batch *Alo, const sell_bv *B, sell_bv *X, double tol,
                  int64_t maxit, double inner_tol, int64_t inner_maxit, uint32_t flags,
                  sell_cg_stats *stats, void *stream);

/* ------------------------------------------------------------------------------------ */
/* Measurement helpers                                                                  */

/* Streaming probes of achievable device bandwidth on caller-owned device buffers:
 *   kind 0: copy  dst[i] = src[i], nontemporal loads and stores   (2 * bytes moved)
 *   kind 1: read  sum of src (nontemporal loads); dst must hold 1 KiB (bytes moved)
 *   kind 2: write dst[i] = constant, nontemporal stores           (bytes moved)
 *   kind 3: copy with ordinary loads and stores                    (2 * bytes moved)
 *   kind 4: write with ordinary stores                             (bytes moved)
 * bytes must be a positive multiple of 16; both buffers 16-byte aligned; src is not read
 * by kinds 2 and 4 (may be NULL). Asynchronous. */
int sell_probe_bandwidth(int kind, void *dst, const void *src, int64_t bytes, void *stream);

/* Streaming probe of a given read:write mix and launch shape, for the achievable-bandwidth
 * figure against which the products are judged (the roofline reading of Sec. 4.1: a kernel
 * bound by memory traffic is measured against what the memory sustains for that traffic).
 * reads R in 0..4 streams of bytes each, laid out one after another in src (R * bytes);
 * writes W in {0, 1}: with W = 1, dst (bytes) receives element by element the sum of the R
 * read streams (16-byte float4 elements; R = 0 writes a constant); with W = 0 the sums are
 * reduced to one 16-byte partial per workgroup in dst (grid * 16 bytes). unroll in {1, 2, 4, 8}:
 * elements per stream and thread in flight (R * unroll loads); nontemporal != 0 uses
 * nontemporal loads and stores; grid: workgroups of 256 threads, 1..2^20, grid-stride.
 * Moves (R + W) * bytes. bytes a positive multiple of 16, buffers 16-byte aligned.
 * Asynchronous. Errors: SELL_ERR_ARG for any other argument. */
int sell_probe_stream(int reads, int writes, int unroll, int nontemporal, int grid, void *dst, const void *src,
                      int64_t bytes, void *stream);

/* Random-gather probe: for i < count, reads row idx[i] of x (nrows rows of row_bytes bytes,
 * row_bytes in {8, 16, 32, 64, 128, 256}; x 8-byte aligned for 8, else 16-byte aligned), 8
 * gathers in flight per thread; rows of 64, 128 and 256 bytes are split over 2, 4 and 8 lanes
 * (32 bytes each, as the product kernels split a row of x). It gives the achievable rate of the scattered row gathers that a product
 * with scattered column indices performs (a row of X per nonzero; Sec. 5.2 notes that SpMMV
 * gathers whole rows of a row-major block vector).
 * idx: device int32[count] (may be NULL when count is 0); entries outside [0, nrows) read
 * row 0. out: device memory of at least 8 bytes, 8-byte aligned (not normally written).
 * Moves count * (row_bytes + 4) bytes of algorithmic data. Asynchronous.
 * Errors: SELL_ERR_ARG for NULL x or out, NULL idx with count > 0, nrows < 1, count < 0,
 * another row_bytes or a misaligned pointer. */
int sell_probe_gather(const void *x, int64_t nrows, int32_t row_bytes, const int32_t *idx, int64_t count,
                      void *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SELLCS_H */
