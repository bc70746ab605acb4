// build.cpp -- host construction of SELL-C-sigma from CSR (GHOST paper, Sec. 5.1).
//
// The format: rows are cut into chunks of C consecutive rows; inside each window of sigma
// rows the rows are first sorted by their number of nonzeros; a chunk is padded with
// trailing zeros to the length of its longest row, and its entries are stored column by
// column ("diagonal-wise"), so that entry k of the row in slot r of chunk c sits at
// cs[c] + k*C + r. Sorting direction and tie-break are not fixed by the paper; this
// library sorts by descending length and keeps equal lengths in their original order
// (a stable sort), which also puts the longest chunks of a window first.
//
// Padding entries carry column -1 and value 0, so the kernels can skip them exactly
// (no gather, no arithmetic) and the original CSR can be recovered bit for bit.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <numeric>
#include <thread>
#include <utility>

#include "convert.h"
#include "internal.h"

namespace sellcs {

namespace {

template <class F>
void parallel_for(int64_t n, F &&f) {
    unsigned hw = std::thread::hardware_concurrency();
    int64_t nt = std::max<int64_t>(1, std::min<int64_t>(hw ? hw : 1, 16));
    if (n < 65536 || nt == 1) {
        f(int64_t(0), n);
        return;
    }
    std::vector<std::thread> th;
    int64_t step = (n + nt - 1) / nt;
    for (int64_t t = 0; t < nt; ++t) {
        int64_t lo = t * step, hi = std::min(n, lo + step);
        if (lo >= hi) break;
        th.emplace_back([&f, lo, hi] { f(lo, hi); });
    }
    for (auto &t : th) t.join();
}

}  // namespace

uint16_t f64_to_bf16_bits(double v) { return bf16_from_f64(v); }

float bf16_bits_to_f32(uint16_t b) { return f32_from_bf16(b); }

void convert_values(const double *src, int64_t n, int vdt, void *dst) {
    if (vdt == SELL_F64) {
        parallel_for(n, [&](int64_t lo, int64_t hi) {
            std::memcpy(static_cast<double *>(dst) + lo, src + lo, sizeof(double) * (hi - lo));
        });
    } else if (vdt == SELL_F32) {
        float *d = static_cast<float *>(dst);
        parallel_for(n, [&](int64_t lo, int64_t hi) {
            for (int64_t i = lo; i < hi; ++i) d[i] = float(src[i]);
        });
    } else {
        uint16_t *d = static_cast<uint16_t *>(dst);
        parallel_for(n, [&](int64_t lo, int64_t hi) {
            for (int64_t i = lo; i < hi; ++i) d[i] = f64_to_bf16_bits(src[i]);
        });
    }
}

int32_t default_tile_count(int64_t nch) {
    int64_t t = kMaxTiles;
    if (const char *e = std::getenv("SELLCS_TILES")) {
        long v = std::strtol(e, nullptr, 10);
        if (v >= 1 && v <= kMaxTiles) t = v;
    }
    return int32_t(std::max<int64_t>(std::min<int64_t>(nch, t), nch > 0 ? 1 : 0));
}

// Contiguous chunk ranges of about equal cost. A chunk's cost is its stored entries plus
// two units per row slot for the epilogue (reads and writes of y).
void make_tiles(const std::vector<int32_t> &cl, int32_t C, int32_t ntiles,
                std::vector<int32_t> &tiles) {
    const int64_t nch = int64_t(cl.size());
    tiles.assign(size_t(ntiles) + 1, 0);
    if (ntiles == 0) return;
    std::vector<int64_t> pre(size_t(nch) + 1, 0);
    for (int64_t c = 0; c < nch; ++c) pre[c + 1] = pre[c] + int64_t(C) * (int64_t(cl[c]) + 2);
    const int64_t total = pre[nch];
    for (int32_t t = 1; t < ntiles; ++t) {
        // first chunk whose prefix cost reaches t/ntiles of the total
        const long double goal = (long double)total * t / ntiles;
        int64_t c = std::lower_bound(pre.begin(), pre.end(), (int64_t)std::ceil(goal)) - pre.begin();
        c = std::min<int64_t>(std::max<int64_t>(c, tiles[t - 1]), nch);
        tiles[t] = int32_t(c);
    }
    tiles[ntiles] = int32_t(nch);
}

// The products issue a chunk's index loads and gathers in batches of U, every batch whole (a
// partial last batch re-reads its last entry: branches around the loads would split the batch
// and serialise its latency). Per chunk of length L that is ceil(L / U) rounds of U loads, and
// a round costs about kRound loads more in latency. kRound = 13 is what the 128^3 Anderson
// product shows (7 entries per row: batches of 7 take 133.6 us against 140.4 us for 8, a ratio
// of (8 + 13) / (7 + 13)). Batches of 5 and 7 exist for the 5- and 7-entry rows of 2D and 3D
// stencils; other lengths keep 8. The kernels whose lane gathers 32 bytes per entry (FP64
// values and vectors, 4 columns per lane) hold 180 VGPRs with 8-entry batches, two waves per
// SIMD, and 162 or 147 with 7 or 5, three waves: there only 7 and 5 compete (the 4 M-row
// irregular matrix at b = 8, sigma = 1024: 1,435 and 1,335 us against 1,534 us for 8).
int32_t choose_batch_len(const std::vector<int32_t> &cl, bool wide) {
    constexpr double kRound = 13.0;
    int32_t best = 0;
    double best_cost = 0.0;
    for (int32_t u : {8, 7, 5}) {
        if (wide && u == 8) continue;
        double cost = 0.0;
        for (int32_t l : cl) cost += double((l + u - 1) / u) * (u + kRound);
        if (best == 0 || cost < best_cost) {
            best = u;
            best_cost = cost;
        }
    }
    return best;
}

// Default grid of the product launches in waves of resident workgroups: 16 when the chunk
// lengths spread widely (coefficient of variation above 1/2: scattered long rows, whose tiles
// run at different speeds however their entries are balanced), else 1. Sixteen waves reach the
// cap of one fine tile per workgroup on matrices of 4096 chunks or more, so the workgroups that
// run at the same time on an XCD (dispatched in order) work on neighbouring rows and share the
// x rows of their banded columns in its L2. Measured on the 4 M-row irregular matrix (sigma =
// 1024): FP64 b = 8 1104 us with 4 waves, 969 with 8 or 16; BF16 values b = 8 915 / 765; FP64
// b = 1 875 in one wave, 751 in 4, 692 in 16. On stencils more waves only cost (the 100^3
// Laplacian, FP32 values, b = 8: 39.4 us in one wave, 53.5 in 4).
int32_t choose_waves(const std::vector<int32_t> &cl) {
    if (cl.size() < 2) return 1;
    double s = 0.0, s2 = 0.0;
    for (int32_t l : cl) {
        s += l;
        s2 += double(l) * l;
    }
    const double n = double(cl.size()), mean = s / n;
    if (mean <= 0.0) return 1;
    const double var = std::max(0.0, s2 / n - mean * mean);
    return std::sqrt(var) > 0.5 * mean ? 16 : 1;
}

int build_host_sell(HostSell &h, int64_t nrows, int64_t ncols, const int64_t *rowptr,
                    const int32_t *col, const double *val, int32_t C, int64_t sigma, int vdt) {
    if (nrows < 0 || ncols < 0 || nrows >= (int64_t(1) << 31) || ncols >= (int64_t(1) << 31))
        return SELL_ERR_ARG;
    if (C < 1 || C > (1 << 20) || sigma < 1) return SELL_ERR_ARG;
    if (vdt != SELL_F64 && vdt != SELL_F32 && vdt != SELL_BF16) return SELL_ERR_DTYPE;
    if (!rowptr) return SELL_ERR_ARG;
    if (rowptr[0] != 0) return SELL_ERR_ARG;
    {
        std::atomic<bool> bad{false};
        parallel_for(nrows, [&](int64_t lo, int64_t hi) {
            for (int64_t i = lo; i < hi; ++i)
                if (rowptr[i + 1] < rowptr[i]) {
                    bad = true;
                    return;
                }
        });
        if (bad) return SELL_ERR_ARG;
    }
    const int64_t nnz = rowptr[nrows];
    if (nnz > 0 && (!col || !val)) return SELL_ERR_ARG;
    {
        std::atomic<bool> bad{false};
        parallel_for(nnz, [&](int64_t lo, int64_t hi) {
            for (int64_t p = lo; p < hi; ++p)
                if (col[p] < 0 || int64_t(col[p]) >= ncols) {
                    bad = true;
                    return;
                }
        });
        if (bad) return SELL_ERR_ARG;
    }

    h = HostSell();
    h.nrows = nrows;
    h.ncols = ncols;
    h.nnz = nnz;
    h.C = C;
    h.sigma = sigma;
    h.vdt = vdt;
    const int64_t nch = (nrows + C - 1) / C;
    h.nch = nch;
    const int64_t nslots = nch * C;

    // row lengths
    std::vector<int64_t> len(static_cast<size_t>(nrows));
    parallel_for(nrows, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) len[i] = rowptr[i + 1] - rowptr[i];
    });

    // sigma-window sort (descending length, stable)
    std::vector<int32_t> slot_row(static_cast<size_t>(nslots));
    parallel_for(nslots, [&](int64_t lo, int64_t hi) {
        for (int64_t s = lo; s < hi; ++s) slot_row[s] = s < nrows ? int32_t(s) : -1;
    });
    const int64_t win = std::min<int64_t>(sigma, std::max<int64_t>(nrows, 1));
    if (win > 1) {
        const int64_t nwin = (nrows + win - 1) / win;
        parallel_for(nwin, [&](int64_t lo, int64_t hi) {
            for (int64_t w = lo; w < hi; ++w) {
                auto b = slot_row.begin() + w * win;
                auto e = slot_row.begin() + std::min(nrows, (w + 1) * win);
                std::stable_sort(b, e, [&](int32_t a, int32_t c) { return len[a] > len[c]; });
            }
        });
        bool ident = true;
        for (int64_t s = 0; s < nrows && ident; ++s) ident = slot_row[s] == s;
        h.has_perm = !ident;
    }

    // chunk lengths (in parallel) and starts (a prefix sum)
    h.cl.assign(size_t(nch), 0);
    h.cs.assign(size_t(nch) + 1, 0);
    std::vector<int64_t> clen(static_cast<size_t>(nch));
    parallel_for(nch, [&](int64_t lo, int64_t hi) {
        for (int64_t c = lo; c < hi; ++c) {
            int64_t m = 0;
            for (int32_t r = 0; r < C; ++r) {
                const int32_t row = slot_row[c * C + r];
                if (row >= 0) m = std::max(m, len[row]);
            }
            clen[c] = m;
        }
    });
    for (int64_t c = 0; c < nch; ++c) {
        if (clen[c] >= (int64_t(1) << 31)) return SELL_ERR_ARG;
        h.cl[c] = int32_t(clen[c]);
        h.cs[c + 1] = h.cs[c] + int64_t(C) * clen[c];
    }
    h.stored = h.cs[nch];

    // column-major fill, padding (col -1, value 0) written in the same pass; values are
    // converted to the storage type on the way (round to nearest even from the double)
    h.col.resize(size_t(h.stored));
    h.val.resize(size_t(h.stored) * dtype_bytes(vdt));
    auto fill = [&](auto *dst, auto conv) {
        parallel_for(nch, [&](int64_t lo, int64_t hi) {
            for (int64_t c = lo; c < hi; ++c)
                for (int32_t r = 0; r < C; ++r) {
                    const int32_t row = slot_row[c * C + r];
                    const int64_t n = row >= 0 ? len[row] : 0;
                    const int64_t p0 = row >= 0 ? rowptr[row] : 0;
                    for (int64_t k = 0; k < h.cl[c]; ++k) {
                        const int64_t at = h.cs[c] + k * C + r;
                        const bool real = k < n;
                        h.col[at] = real ? col[p0 + k] : -1;
                        dst[at] = conv(real ? val[p0 + k] : 0.0);
                    }
                }
        });
    };
    if (vdt == SELL_F64)
        fill(reinterpret_cast<double *>(h.val.data()), [](double v) { return v; });
    else if (vdt == SELL_F32)
        fill(reinterpret_cast<float *>(h.val.data()), [](double v) { return float(v); });
    else
        fill(reinterpret_cast<uint16_t *>(h.val.data()), [](double v) { return f64_to_bf16_bits(v); });

    if (h.has_perm) h.perm = std::move(slot_row);
    h.rowptr.assign(rowptr, rowptr + nrows + 1);
    const int32_t nt = default_tile_count(nch);
    make_tiles(h.cl, C, nt, h.tiles);
    h.batch = choose_batch_len(h.cl);
    h.batch_wide = choose_batch_len(h.cl, true);
    h.waves = choose_waves(h.cl);
    return SELL_OK;
}

}  // namespace sellcs
