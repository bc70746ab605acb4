// tune.cpp -- choice of the SELL-C-sigma parameters and launch shape by timed trials.
//
// The paper picks C from the hardware (the SIMD width or the warp size) and sigma as a
// compromise between padding and the locality of the right-hand side (Sec. 5.1), and plans
// micro-benchmarks for decisions that depend on the device (Sec. 7.2). Here the candidates are
// timed on the device itself: first (C, sigma) pairs with the default launch, then, for the
// best pair, the columns per lane of the fixed-width kernels, the workgroups per compute unit
// and the grid size in waves of resident workgroups. Each trial times the augmented product that a CG iteration issues (y = A x with the
// fused <x, y>, or the plain product for a rectangular matrix) with HIP events.
//
// The default (C = 32, sigma = 1, default launch) is timed first; a candidate must beat the best
// so far by 3 % to replace it. A last stage times the block in slices of 8, 16 or 32 columns
// (several launches of a narrower width can beat one wide launch).
//
// Results are cached for the process under a key that describes the matrix's shape class: the
// value type, the block width, the binary order of magnitude of the row count, the mean row
// length and the histogram of row lengths over power-of-two bins (fractions rounded to 1/32).
// Matrices of one family and similar size therefore share one tuning run.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "log.h"

using namespace sellcs;

namespace {

#define HIPCHK(x)                                                                             \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess) return e_ == hipErrorOutOfMemory ? SELL_ERR_OOM : SELL_ERR_HIP; \
    } while (0)

// A candidate replaces the best so far only when it is faster by more than the timing noise, so
// matrices of one family do not end up with different choices of equal speed.
constexpr double kMargin = 0.97;

std::mutex g_mu;
std::map<std::string, sell_tune_result> g_cache;

std::string shape_key(int64_t nrows, int64_t ncols, const int64_t *rowptr, int vdt, int b) {
    std::vector<int64_t> hist(34, 0);
    for (int64_t i = 0; i < nrows; ++i) {
        const int64_t len = rowptr[i + 1] - rowptr[i];
        int bin = 0;
        while (bin < 33 && (int64_t(1) << bin) <= len) ++bin;  // 0: empty, k: [2^(k-1), 2^k)
        hist[size_t(bin)]++;
    }
    std::string key = std::to_string(vdt) + "/" + std::to_string(b) + "/" + (nrows == ncols ? "sq" : "rect") + "/";
    int mag = 0;
    while ((int64_t(1) << mag) < nrows) ++mag;
    key += std::to_string(mag) + "/";
    const double mean = nrows > 0 ? double(rowptr[nrows] - rowptr[0]) / double(nrows) : 0.0;
    key += std::to_string(int(std::lround(mean * 2))) + "/";
    for (int64_t h : hist) key += std::to_string(nrows > 0 ? std::lround(32.0 * double(h) / double(nrows)) : 0) + ",";
    return key;
}

struct Trial {
    int32_t C;
    int64_t sigma;
    int32_t vpt, bpc;
    double us;
    int32_t slice = 0;
    int32_t waves = 0;
    int32_t batch = 0;
};

// Average time of one product on A (after warm-up launches).
int time_product(sell_mat *A, const sell_bv *X, sell_bv *Y, double *dot, int reps, hipStream_t s, double *us) {
    sell_spmv_opts o = SELL_SPMV_OPTS_INIT;
    const bool square = A->h.nrows == A->h.ncols;
    o.flags = square ? SELL_SPMV_DOT_XY : 0;
    o.dot = dot;
    int rc;
    for (int w = 0; w < 3; ++w)
        if ((rc = aug_impl(A, X, Y, nullptr, o, square, s))) return rc;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return SELL_ERR_HIP;
    }
    rc = SELL_OK;
    if (hipEventRecord(e0, s) != hipSuccess) rc = SELL_ERR_HIP;
    for (int r = 0; r < reps && rc == SELL_OK; ++r) rc = aug_impl(A, X, Y, nullptr, o, square, s);
    if (rc == SELL_OK && hipEventRecord(e1, s) != hipSuccess) rc = SELL_ERR_HIP;
    float ms = 0.f;
    if (rc == SELL_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = SELL_ERR_HIP;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *us = 1000.0 * double(ms) / reps;
    return rc;
}

}  // namespace

extern "C" {

int sell_set_launch(sell_mat *A, int32_t vpt, int32_t blocks_per_cu) {
    if (!A) return SELL_ERR_ARG;
    if (!(vpt == 0 || vpt == 1 || vpt == 2 || vpt == 4)) return SELL_ERR_ARG;
    if (blocks_per_cu < 0 || blocks_per_cu > 64) return SELL_ERR_ARG;
    A->vpt_hint = vpt;
    A->bpc_hint = blocks_per_cu;
    return SELL_OK;
}

int sell_set_waves(sell_mat *A, int32_t waves) {
    if (!A) return SELL_ERR_ARG;
    if (!(waves == 0 || waves == 1 || waves == 2 || waves == 4 || waves == 8 || waves == 16)) return SELL_ERR_ARG;
    A->waves_hint = waves;
    return SELL_OK;
}

int sell_set_batch(sell_mat *A, int32_t batch) {
    if (!A) return SELL_ERR_ARG;
    if (!(batch == 0 || batch == 5 || batch == 7 || batch == 8)) return SELL_ERR_ARG;
    A->batch_hint = batch;
    return SELL_OK;
}

int sell_set_stage(sell_mat *A, int32_t stage, int32_t tile_stride) {
    if (!A) return SELL_ERR_ARG;
    if (stage < 0 || stage > 1 || tile_stride < 0) return SELL_ERR_ARG;
    A->stage_hint = stage;
    A->tile_stride_hint = tile_stride;
    return SELL_OK;
}

int sell_set_slice(sell_mat *A, int32_t slice) {
    if (!A) return SELL_ERR_ARG;
    if (!(slice == 0 || slice == 1 || slice == 2 || slice == 4 || slice == 8 || slice == 16 || slice == 32))
        return SELL_ERR_ARG;
    A->slice_hint = slice;
    return SELL_OK;
}

int sell_autotune(int64_t nrows, int64_t ncols, const int64_t *rowptr, const int32_t *col, const double *val,
                  sell_dtype vdt, int32_t b, uint32_t flags, sell_tune_result *out, void *stream) {
    if (!out || !rowptr || nrows < 0 || ncols < 0) return SELL_ERR_ARG;
    if (b < 1 || b > kMaxSliceCols) return SELL_ERR_UNSUPPORTED;
    if (flags & ~uint32_t(SELL_TUNE_NO_CACHE)) return SELL_ERR_ARG;
    if (vdt != SELL_F64 && vdt != SELL_F32 && vdt != SELL_BF16) return SELL_ERR_DTYPE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::string key;
    try {
        key = shape_key(nrows, ncols, rowptr, int(vdt), b);
    } catch (...) {
        return SELL_ERR_OOM;
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_cache.find(key);
        if (!(flags & SELL_TUNE_NO_CACHE) && it != g_cache.end()) {
            *out = it->second;
            out->trials = 0;
            return SELL_OK;
        }
    }
    // operands of the trials: X = 1, Y = 0 in the matrix's vector type
    const int vt = vdt == SELL_F64 ? SELL_F64 : SELL_F32;
    const size_t es = vt == SELL_F64 ? 8 : 4;
    void *px = nullptr, *py = nullptr;
    double *pdot = nullptr;
    HIPCHK(lib_malloc(&px, std::max<size_t>(16, size_t(ncols) * b * es)));
    auto cleanup = [&]() {
        if (px) (void)lib_free(px);
        if (py) (void)lib_free(py);
        if (pdot) (void)lib_free(pdot);
    };
    if (lib_malloc(&py, std::max<size_t>(16, size_t(nrows) * b * es)) != hipSuccess ||
        lib_malloc(reinterpret_cast<void **>(&pdot), 3 * kMaxSliceCols * sizeof(double)) != hipSuccess) {
        cleanup();
        return SELL_ERR_OOM;
    }
    int rc = launch_fill(px, vt, ncols, b, b, 1, 1.0, s);
    if (!rc) rc = launch_fill(py, vt, nrows, b, b, 1, 0.0, s);
    sell_bv X, Y;
    X.nrows = ncols;
    X.ncols = b;
    X.dt = vt;
    X.lay = SELL_ROW_MAJOR;
    X.ptr = px;
    X.ld = b;
    Y = X;
    Y.nrows = nrows;
    Y.ptr = py;

    std::vector<Trial> trials;
    const int reps = 10;
    auto run = [&](int32_t C, int64_t sigma, int32_t vpt, int32_t bpc, sell_mat *reuse, Trial *res) -> int {
        sell_mat *A = reuse;
        int r = SELL_OK;
        if (!A && (r = sell_build(&A, nrows, ncols, rowptr, col, val, C, sigma, vdt, s))) return r;
        A->vpt_hint = vpt;
        A->bpc_hint = bpc;
        double us = 0.0;
        r = time_product(A, &X, &Y, pdot, reps, s, &us);
        if (!reuse) sell_destroy(A);
        if (r) return r;
        *res = Trial{C, sigma, vpt, bpc, us};
        trials.push_back(*res);
        return SELL_OK;
    };

    // stage 1: (C, sigma) with the default launch, the default pair first
    std::vector<std::pair<int32_t, int64_t>> pairs{{32, 1}};
    for (int32_t C : {16, 32, 64}) {
        const int64_t sigmas[] = {1, 8 * int64_t(C), 256 * int64_t(C)};
        for (int64_t sg : sigmas) {
            if (C == 32 && sg == 1) continue;
            if (sg > 1 && sg >= nrows && sg != sigmas[1]) continue;  // one whole-matrix window suffices
            pairs.emplace_back(C, sg);
        }
    }
    Trial best{32, 1, 0, 0, INFINITY}, deflt{32, 1, 0, 0, INFINITY};
    for (const auto &cs : pairs) {
        if (rc) break;
        Trial t;
        rc = run(cs.first, cs.second, 0, 0, nullptr, &t);
        if (rc) break;
        if (cs.first == 32 && cs.second == 1) deflt = t;
        if (t.us < kMargin * best.us) best = t;
    }
    // stage 2: launch shape for the best pair
    if (!rc) {
        sell_mat *A = nullptr;
        rc = sell_build(&A, nrows, ncols, rowptr, col, val, best.C, best.sigma, vdt, s);
        if (!rc) {
            std::vector<int32_t> vpts;
            for (int v : {1, 2, 4})
                if (v <= b && (b == 1 || b == 2 || b == 4 || b == 8 || b == 16 || b == 32)) vpts.push_back(v);
            for (int32_t v : vpts)
                for (int32_t bpc : {0, 1, 2}) {
                    if (rc) break;
                    if (v == choose_vpt(vdt == SELL_F64 ? VK_F64F64 : VK_F32F32, b) && bpc == 0) continue;  // stage 1
                    Trial t;
                    rc = run(best.C, best.sigma, v, bpc, A, &t);
                    if (!rc && t.us < kMargin * best.us) best = t;
                }
            // grids of several waves of resident workgroups (uneven tiles balance dynamically)
            for (int32_t wv : {1, 2, 4, 8}) {
                if (rc) break;
                if (wv == std::max(A->h.waves, 1)) continue;  // the default grid, timed above
                A->waves_hint = wv;
                Trial t;
                rc = run(best.C, best.sigma, best.vpt, best.bpc, A, &t);
                A->waves_hint = 0;
                t.waves = wv;
                if (!rc) {
                    trials.back().waves = wv;
                    if (t.us < kMargin * best.us) best = t;
                }
            }
            // index batch lengths set for every kernel (against the construction's choice)
            for (int32_t bl : {5, 7, 8}) {
                if (rc) break;
                A->batch_hint = bl;
                A->waves_hint = best.waves;
                Trial t;
                rc = run(best.C, best.sigma, best.vpt, best.bpc, A, &t);
                A->batch_hint = 0;
                A->waves_hint = 0;
                t.waves = best.waves;
                t.batch = bl;
                if (!rc) {
                    trials.back().waves = best.waves;
                    trials.back().batch = bl;
                    if (t.us < kMargin * best.us) best = t;
                }
            }
            // stage 3: the block in slices of 8, 16 or 32 columns (the b packing), timed as the
            // whole sliced call with the best launch shape
            for (int32_t sl : {8, 16, 32}) {
                if (rc || sl >= b || b % sl != 0) continue;
                A->slice_hint = sl;
                A->waves_hint = best.waves;
                A->batch_hint = best.batch;
                Trial t;
                rc = run(best.C, best.sigma, best.vpt, best.bpc, A, &t);
                A->slice_hint = 0;
                A->waves_hint = 0;
                A->batch_hint = 0;
                t.slice = sl;
                t.waves = best.waves;
                t.batch = best.batch;
                if (!rc) {
                    trials.back().slice = sl;
                    trials.back().waves = best.waves;
                    trials.back().batch = best.batch;
                    if (t.us < kMargin * best.us) best = t;
                }
            }
            sell_destroy(A);
        }
    }
    cleanup();
    if (rc) return rc;
    sell_tune_result res;
    res.C = best.C;
    res.sigma = best.sigma;
    res.vpt = best.vpt;
    res.blocks_per_cu = best.bpc;
    res.slice = best.slice;
    res.waves = best.waves;
    res.batch = best.batch;
    res.us = best.us;
    res.default_us = deflt.us;
    res.trials = int32_t(trials.size());
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_cache[key] = res;
    }
    log_info("autotune %lld x %lld, b = %d: C = %d, sigma = %lld, %d columns per lane, %d workgroup(s) per CU, "
             "slice %d, %d wave(s), index batch %d: %.1f us against %.1f us for SELL-32-1 (%d trials)",
             (long long)nrows, (long long)ncols, int(b), int(res.C), (long long)res.sigma, int(res.vpt),
             int(res.blocks_per_cu), int(res.slice), int(res.waves), int(res.batch), res.us, res.default_us,
             int(res.trials));
    *out = res;
    return SELL_OK;
}

}  // extern "C"
