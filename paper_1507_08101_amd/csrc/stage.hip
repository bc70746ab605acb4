// stage.hip -- per-tile page lists of x and tile-local column indices for the product kernels
// that gather x through LDS.
//
// The rows of x (the block vector the product gathers from) are grouped in pages of
// kStagePage consecutive rows. For every work tile (a contiguous chunk range), this builds the
// sorted list of the pages its entries reference, if there are at most kStageMaxPages of them,
// and re-expresses every stored column index of the tile as (position of its page in that
// list, row within the page) in 16 bits. A workgroup then loads the tile's pages into LDS once
// and gathers from there; pages that the previous tile of the same workgroup already loaded
// stay. This is the compression of column indices that the row-wise distribution of a matrix
// applies to the columns a process reads from others (Sec. 4.1), applied to the x rows that one
// workgroup holds at a time.
#include <mutex>

#include "internal.h"

namespace sellcs {

namespace {

constexpr int kT = 512;
constexpr int kHash = 2048;  // open-addressing table of distinct pages (power of two)

// One workgroup per stage tile (chunks consecutive chunks; the last one may be shorter).
// np[t]: number of pages (0: the tile is not staged: no entries, or more than
// kStageMaxPages pages); pages[t * kStageMaxPages + i]: the i-th page, ascending;
// own[t]: position in that list of the page of the tile's first row when every row of the
// tile (slots without a permutation) lies in a listed page, else -1;
// lcol[e]: position << kStagePageShift | (column & (kStagePage - 1)), 0xFFFF for padding.
__global__ void __launch_bounds__(kT) stage_build_kernel(const int32_t *__restrict__ col, const int64_t *__restrict__ cs,
                                                        int64_t nch, int32_t chunks, int32_t C, int64_t nrows,
                                                        int has_perm, int32_t *__restrict__ np,
                                                        int32_t *__restrict__ pages, int32_t *__restrict__ own,
                                                        uint16_t *__restrict__ lcol) {
    __shared__ int32_t table[kHash];
    __shared__ int32_t list[kStageMaxPages];
    __shared__ int32_t sorted[kStageMaxPages];
    __shared__ int32_t count, overflow, fill;
    const int t = blockIdx.x, tid = threadIdx.x;
    const int64_t c0 = int64_t(t) * chunks, c1 = c0 + chunks < nch ? c0 + chunks : nch;
    const int64_t e0 = cs[c0], e1 = cs[c1];
    for (int i = tid; i < kHash; i += kT) table[i] = -1;
    if (tid == 0) {
        count = 0;
        overflow = 0;
        fill = 0;
    }
    __syncthreads();
    for (int64_t e = e0 + tid; e < e1; e += kT) {
        if (*reinterpret_cast<volatile int32_t *>(&overflow)) break;
        const int32_t c = col[e];
        if (c < 0) continue;
        const int32_t p = c >> kStagePageShift;
        uint32_t h = (uint32_t(p) * 2654435761u) & (kHash - 1);
        for (int probe = 0;; ++probe) {
            if (probe == kHash) {  // cannot happen below kStageMaxPages distinct pages; bounded anyway
                atomicExch(&overflow, 1);
                break;
            }
            const int32_t old = atomicCAS(&table[h], -1, p);
            if (old == -1) {
                if (atomicAdd(&count, 1) >= kStageMaxPages) atomicExch(&overflow, 1);
                break;
            }
            if (old == p) break;
            h = (h + 1) & (kHash - 1);
        }
    }
    __syncthreads();
    const int n = count;
    if (overflow || n == 0 || n > kStageMaxPages) {
        if (tid == 0) {
            np[t] = 0;
            own[t] = -1;
        }
        return;  // uniform: the tile keeps its global column indices
    }
    for (int i = tid; i < kHash; i += kT) {
        const int32_t p = table[i];
        if (p >= 0) list[atomicAdd(&fill, 1)] = p;
    }
    __syncthreads();
    if (tid < n) {  // rank sort of distinct values
        const int32_t p = list[tid];
        int r = 0;
        for (int j = 0; j < n; ++j) r += list[j] < p;
        sorted[r] = p;
    }
    __syncthreads();
    if (tid < n) pages[int64_t(t) * kStageMaxPages + tid] = sorted[tid];
    if (tid == 0) {
        np[t] = n;
        // own rows: slot == row without a permutation; the tile's rows are [r0, r1)
        int32_t o = -1;
        if (!has_perm) {
            const int64_t r0 = c0 * C;
            int64_t r1 = c1 * C;
            if (r1 > nrows) r1 = nrows;
            if (r1 > r0) {
                const int32_t p0 = int32_t(r0 >> kStagePageShift), p1 = int32_t((r1 - 1) >> kStagePageShift);
                int pos = -1;
                for (int j = 0; j < n; ++j)
                    if (sorted[j] == p0) pos = j;
                // the pages of the rows are consecutive ids, so they must be consecutive entries
                if (pos >= 0 && pos + (p1 - p0) < n && sorted[pos + (p1 - p0)] == p1) o = pos;
            }
        }
        own[t] = o;
    }
    for (int64_t e = e0 + tid; e < e1; e += kT) {
        const int32_t c = col[e];
        uint16_t l = 0xFFFFu;
        if (c >= 0) {
            const int32_t p = c >> kStagePageShift;
            int lo = 0, hi = n - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (sorted[mid] < p)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            l = uint16_t((lo << kStagePageShift) | (c & (kStagePage - 1)));
        }
        lcol[e] = l;
    }
}

// One thread per workgroup of a staged launch (nblk workgroups, unit stride S): walks the
// workgroup's units in the kernel's order and fixes, for every staged unit, the cache slot of
// each of its pages (slot[u * kStageMaxPages + i]) and the pages it must load (bit i of
// miss[u]). It follows the kernel's rule: the pages of a unit are loaded during the unit
// before it when both units' pages fit in the ns slots together (the earlier unit's pages
// stay), else after it; the first unit's before any work. Missing pages take the lowest free
// slots.
__global__ void stage_plan_kernel(const int32_t *__restrict__ np, const int32_t *__restrict__ pages, int64_t nunits,
                                  int nblk, int S, int ns, int8_t *__restrict__ slot, uint64_t *__restrict__ miss) {
    const int g = int(blockIdx.x) * int(blockDim.x) + int(threadIdx.x);
    if (g >= nblk) return;
    int64_t r_first, r_count, r_step;
    if (S > 0) {
        const int64_t Q = nunits / S, nseg = nblk / S, q = g / S;
        const int64_t k0 = q * Q / nseg, k1 = (q + 1) * Q / nseg;
        r_first = (g % S) + S * k0;
        r_count = k1 - k0;
        r_step = S;
    } else {
        const int64_t t0 = int64_t(g) * nunits / nblk, t1 = int64_t(g + 1) * nunits / nblk;
        r_first = t0;
        r_count = t1 - t0;
        r_step = 1;
    }
    int32_t tag[kStageMaxPages];
    bool keep[kStageMaxPages];
    for (int j = 0; j < ns; ++j) tag[j] = -1;
    auto listed = [&](int64_t u, int n, int32_t p) {  // binary search in unit u's sorted pages
        int lo = 0, hi = n - 1;
        while (lo <= hi) {
            const int mid = (lo + hi) >> 1;
            const int32_t v = pages[u * kStageMaxPages + mid];
            if (v == p) return true;
            if (v < p)
                lo = mid + 1;
            else
                hi = mid - 1;
        }
        return false;
    };
    int prev_n = 0;
    int64_t prev = -1;
    for (int64_t k = 0; k < r_count; ++k) {
        const int64_t u = r_first + k * r_step;
        int n = np[u];
        n = (n > 0 && n <= ns) ? n : 0;
        if (n > 0) {
            const bool keep_prev = k > 0 && prev_n + n <= ns;
            for (int j = 0; j < ns; ++j) {
                const int32_t t = tag[j];
                keep[j] = t >= 0 && (listed(u, n, t) || (keep_prev && prev_n > 0 && listed(prev, prev_n, t)));
            }
            uint64_t m = 0;
            int cursor = 0;
            for (int i = 0; i < n; ++i) {
                const int32_t p = pages[u * kStageMaxPages + i];
                int sl = -1;
                for (int j = 0; j < ns; ++j)
                    if (tag[j] == p) sl = j;
                if (sl < 0) {
                    while (keep[cursor]) ++cursor;  // a free slot exists: the kept pages and n fit
                    sl = cursor;
                    keep[sl] = true;
                    tag[sl] = p;
                    m |= uint64_t(1) << i;
                }
                slot[u * kStageMaxPages + i] = int8_t(sl);
            }
            miss[u] = m;
        }
        prev_n = n;
        prev = u;
    }
}

std::mutex g_stage_mu;

}  // namespace

int ensure_stage(const sell_mat *A0, int32_t chunks, hipStream_t s) {
    sell_mat *A = const_cast<sell_mat *>(A0);
    std::lock_guard<std::mutex> lk(g_stage_mu);
    if (chunks < 1 || A->h.nch <= 0) return SELL_ERR_ARG;
    if (A->d_lcol && A->stage_chunks == chunks) return SELL_OK;
    const int64_t nst = (A->h.nch + chunks - 1) / chunks;
    if (nst > INT32_MAX) return SELL_ERR_UNSUPPORTED;
    const size_t nt = size_t(nst);
    int32_t *np = nullptr, *pages = nullptr, *own = nullptr;
    uint16_t *lcol = nullptr;
    hipError_t e = lib_malloc(&np, nt * sizeof(int32_t));
    if (e == hipSuccess) e = lib_malloc(&pages, nt * kStageMaxPages * sizeof(int32_t));
    if (e == hipSuccess) e = lib_malloc(&own, nt * sizeof(int32_t));
    if (e == hipSuccess) e = lib_malloc(&lcol, size_t(std::max<int64_t>(A->h.stored, 1)) * sizeof(uint16_t));
    if (e == hipSuccess) {
        hipLaunchKernelGGL(stage_build_kernel, dim3(unsigned(nst)), dim3(kT), 0, s, A->d_col, A->d_cs, A->h.nch, chunks,
                           A->h.C, A->h.nrows, A->d_perm ? 1 : 0, np, pages, own, lcol);
        e = hipGetLastError();
    }
    // the arrays are read by later launches on any stream: finish building them here
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        lib_free(np);
        lib_free(pages);
        lib_free(own);
        lib_free(lcol);
        return e == hipErrorOutOfMemory ? SELL_ERR_OOM : SELL_ERR_HIP;
    }
    // the previous tile size's arrays are no longer used by any launch (callers order their
    // streams; the build synchronised this one)
    lib_free(A->d_stage_np);
    lib_free(A->d_stage_pages);
    lib_free(A->d_stage_own);
    lib_free(A->d_lcol);
    lib_free(A->d_plan_slot);
    lib_free(A->d_plan_miss);
    A->d_plan_slot = nullptr;
    A->d_plan_miss = nullptr;
    A->d_stage_np = np;
    A->d_stage_pages = pages;
    A->d_stage_own = own;
    A->d_lcol = lcol;
    A->stage_chunks = chunks;
    A->stage_ntiles = int32_t(nst);
    A->plan_nblk = A->plan_stride = A->plan_ns = -1;  // any plan was for the old units
    return SELL_OK;
}

int ensure_stage_plan(const sell_mat *A0, int32_t nblk, int32_t stride, int32_t ns, hipStream_t s) {
    sell_mat *A = const_cast<sell_mat *>(A0);
    std::lock_guard<std::mutex> lk(g_stage_mu);
    if (!A->d_lcol || nblk < 1 || ns < 1 || ns > kStageMaxPages) return SELL_ERR_ARG;
    if (A->d_plan_slot && A->plan_nblk == nblk && A->plan_stride == stride && A->plan_ns == ns) return SELL_OK;
    const size_t nt = size_t(A->stage_ntiles);
    int8_t *slot = A->d_plan_slot;
    uint64_t *miss = A->d_plan_miss;
    hipError_t e = hipSuccess;
    if (!slot) e = lib_malloc(&slot, nt * kStageMaxPages);
    if (e == hipSuccess && !miss) e = lib_malloc(&miss, nt * sizeof(uint64_t));
    if (e == hipSuccess) {
        hipLaunchKernelGGL(stage_plan_kernel, dim3(unsigned((nblk + 63) / 64)), dim3(64), 0, s, A->d_stage_np,
                           A->d_stage_pages, int64_t(A->stage_ntiles), nblk, stride, ns, slot, miss);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    A->d_plan_slot = slot;  // kept (sized by the units) even when the plan failed
    A->d_plan_miss = miss;
    if (e != hipSuccess) {
        A->plan_nblk = -1;
        return e == hipErrorOutOfMemory ? SELL_ERR_OOM : SELL_ERR_HIP;
    }
    A->plan_nblk = nblk;
    A->plan_stride = stride;
    A->plan_ns = ns;
    return SELL_OK;
}

}  // namespace sellcs
