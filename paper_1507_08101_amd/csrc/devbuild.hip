// devbuild.hip -- construction of SELL-C-sigma on the device from a CSR matrix that is already
// in device memory (GHOST paper, Sec. 5.1: the format, the sigma-window sort, padding to the
// chunk's longest row, column-major storage inside a chunk).
//
// The steps are the host builder's, as device kernels and library primitives, and the result
// is identical to it entry for entry:
//   row lengths; inside each window of sigma rows a stable sort by descending length (a stable
//   radix sort of the 64-bit keys (window, 2^31 - 1 - length), which keeps equal keys in row
//   order); chunk lengths as the maximum over the chunk's slots; chunk starts as an exclusive
//   prefix sum of C * length; one thread per slot writes its row's entries and its padding
//   (column -1, value 0), converted to the storage type.
// The small per-chunk arrays, the permutation and the row pointers are copied back to the host
// (the matrix keeps them there, as a host-built one does), where the work partition is made.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <vector>

#include "convert.h"
#include "internal.h"

namespace sellcs {

namespace {

constexpr int kT = 256;

unsigned grid_for(int64_t n) {
    int64_t g = (n + kT - 1) / kT;
    if (g < 1) g = 1;
    if (g > 65535) g = 65535;
    return unsigned(g);
}

// flags[0] = 1 when the row pointers decrease or a row is 2^31 entries or longer;
// flags[1] = 1 when a column index is out of range. Plain stores of the same value.
__global__ void __launch_bounds__(kT) check_kernel(const int64_t *rowptr, const int32_t *col, int64_t nrows,
                                                   int64_t ncols, int64_t nnz, int32_t *flags) {
    const int64_t stride = int64_t(gridDim.x) * kT;
    for (int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x; i < nrows; i += stride) {
        const int64_t d = rowptr[i + 1] - rowptr[i];
        if (d < 0 || d >= (int64_t(1) << 31)) flags[0] = 1;
    }
    for (int64_t p = int64_t(blockIdx.x) * kT + threadIdx.x; p < nnz; p += stride) {
        const int32_t c = col[p];
        if (c < 0 || int64_t(c) >= ncols) flags[1] = 1;
    }
}

// len[i] = row length; with sorting, the key (window, 2^31 - 1 - length) and the row index.
__global__ void __launch_bounds__(kT) lengths_kernel(const int64_t *rowptr, int64_t nrows, int64_t sigma,
                                                     int32_t *len, uint64_t *keys, int32_t *rows) {
    for (int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x; i < nrows; i += int64_t(gridDim.x) * kT) {
        const int32_t l = int32_t(rowptr[i + 1] - rowptr[i]);
        len[i] = l;
        if (keys) {
            keys[i] = (uint64_t(i / sigma) << 32) | uint64_t(uint32_t(0x7fffffff - l));
            rows[i] = int32_t(i);
        }
    }
}

// slot -> row for the slots past the sorted rows (-1), and flags[2] = 1 when a slot holds
// another row than its own index.
__global__ void __launch_bounds__(kT) perm_tail_kernel(int32_t *slot_row, int64_t nrows, int64_t nslots,
                                                       int32_t *flags) {
    for (int64_t s = int64_t(blockIdx.x) * kT + threadIdx.x; s < nslots; s += int64_t(gridDim.x) * kT) {
        if (s >= nrows)
            slot_row[s] = -1;
        else if (slot_row[s] != int32_t(s))
            flags[2] = 1;
    }
}

// cl[c] = the longest row of chunk c; csz[c] = C * cl[c] (csz[nch] = 0 for the prefix sum).
__global__ void __launch_bounds__(kT) chunk_len_kernel(const int32_t *len, const int32_t *slot_row, int64_t nrows,
                                                       int64_t nch, int32_t C, int32_t *cl, int64_t *csz) {
    for (int64_t c = int64_t(blockIdx.x) * kT + threadIdx.x; c <= nch; c += int64_t(gridDim.x) * kT) {
        if (c == nch) {
            csz[c] = 0;
            continue;
        }
        int32_t m = 0;
        for (int32_t r = 0; r < C; ++r) {
            const int64_t s = c * C + r;
            const int64_t row = slot_row ? int64_t(slot_row[s]) : (s < nrows ? s : -1);
            if (row >= 0) m = max(m, len[row]);
        }
        cl[c] = m;
        csz[c] = int64_t(C) * m;
    }
}

// One thread per slot: the row's entries and the padding of its chunk column.
template <class V>
__global__ void __launch_bounds__(kT) fill_kernel(const int64_t *rowptr, const int32_t *col_in,
                                                  const double *val_in, const int32_t *len, const int32_t *slot_row,
                                                  const int32_t *cl, const int64_t *cs, int64_t nrows, int64_t nslots,
                                                  int32_t C, int32_t *col, V *val) {
    for (int64_t s = int64_t(blockIdx.x) * kT + threadIdx.x; s < nslots; s += int64_t(gridDim.x) * kT) {
        const int64_t c = s / C, r = s - c * C;
        const int64_t row = slot_row ? int64_t(slot_row[s]) : (s < nrows ? s : -1);
        const int32_t n = row >= 0 ? len[row] : 0;
        const int64_t p0 = row >= 0 ? rowptr[row] : 0;
        const int32_t m = cl[c];
        const int64_t base = cs[c] + r;
        for (int32_t k = 0; k < m; ++k) {
            const bool real = k < n;
            col[base + int64_t(k) * C] = real ? col_in[p0 + k] : -1;
            val[base + int64_t(k) * C] = Conv<V, double>::go(real ? val_in[p0 + k] : 0.0);
        }
    }
}

struct DevTemp {
    std::vector<void *> p;
    ~DevTemp() {
        for (void *q : p) (void)lib_free(q);
    }
    hipError_t alloc(void **q, size_t bytes) {
        *q = nullptr;
        hipError_t e = lib_malloc(q, bytes ? bytes : 16);
        if (e == hipSuccess) p.push_back(*q);
        return e;
    }
};

int herr(hipError_t e) { return e == hipErrorOutOfMemory ? SELL_ERR_OOM : SELL_ERR_HIP; }

}  // namespace

// Builds into M (fresh, not yet on the device). Returns SELL_OK or an error; on error the
// caller frees whatever device arrays M holds.
int build_device_sell(sell_mat *M, int64_t nrows, int64_t ncols, const int64_t *rowptr, const int32_t *col,
                      const double *val, int32_t C, int64_t sigma, int vdt, hipStream_t s) {
#define DCHK(x)                                  \
    do {                                         \
        hipError_t e_ = (x);                     \
        if (e_ != hipSuccess) return herr(e_);   \
    } while (0)
    HostSell &h = M->h;
    if (nrows < 0 || ncols < 0 || nrows >= (int64_t(1) << 31) || ncols >= (int64_t(1) << 31)) return SELL_ERR_ARG;
    if (C < 1 || C > (1 << 20) || sigma < 1) return SELL_ERR_ARG;
    if (vdt != SELL_F64 && vdt != SELL_F32 && vdt != SELL_BF16) return SELL_ERR_DTYPE;
    if (!rowptr) return SELL_ERR_ARG;
    DCHK(hipGetDevice(&M->device));
    // row pointers to the host (the matrix keeps them), first and last entries checked there
    h = HostSell();
    h.rowptr.resize(size_t(nrows) + 1);
    DCHK(hipMemcpyAsync(h.rowptr.data(), rowptr, sizeof(int64_t) * (size_t(nrows) + 1), hipMemcpyDeviceToHost, s));
    DCHK(hipStreamSynchronize(s));
    if (h.rowptr[0] != 0) return SELL_ERR_ARG;
    const int64_t nnz = h.rowptr[size_t(nrows)];
    if (nnz < 0) return SELL_ERR_ARG;
    if (nnz > 0 && (!col || !val)) return SELL_ERR_ARG;
    const int64_t nch = (nrows + C - 1) / C, nslots = nch * C;
    const int64_t win = std::min<int64_t>(sigma, std::max<int64_t>(nrows, 1));
    const bool sort = win > 1;

    DevTemp T;
    int32_t *flags, *len, *slot_row = nullptr;
    int64_t *csz;
    DCHK(T.alloc(reinterpret_cast<void **>(&flags), 4 * sizeof(int32_t)));
    DCHK(hipMemsetAsync(flags, 0, 4 * sizeof(int32_t), s));
    hipLaunchKernelGGL(check_kernel, dim3(grid_for(std::max(nrows, nnz))), dim3(kT), 0, s, rowptr, col, nrows, ncols,
                       nnz, flags);
    DCHK(hipGetLastError());
    DCHK(T.alloc(reinterpret_cast<void **>(&len), sizeof(int32_t) * size_t(std::max<int64_t>(nrows, 1))));
    uint64_t *keys = nullptr, *keys_out = nullptr;
    int32_t *rows = nullptr;
    if (sort) {
        DCHK(T.alloc(reinterpret_cast<void **>(&keys), sizeof(uint64_t) * size_t(nrows)));
        DCHK(T.alloc(reinterpret_cast<void **>(&keys_out), sizeof(uint64_t) * size_t(nrows)));
        DCHK(T.alloc(reinterpret_cast<void **>(&rows), sizeof(int32_t) * size_t(nrows)));
        DCHK(lib_malloc(reinterpret_cast<void **>(&slot_row), sizeof(int32_t) * size_t(nslots)));
        M->d_perm = slot_row;  // owned by the matrix from here on (freed with it, or dropped below)
    }
    if (nrows > 0) {
        hipLaunchKernelGGL(lengths_kernel, dim3(grid_for(nrows)), dim3(kT), 0, s, rowptr, nrows, win, len, keys, rows);
        DCHK(hipGetLastError());
    }
    int32_t hflags[4] = {0, 0, 0, 0};
    if (sort && nrows > 0) {
        int nwin_bits = 0;
        while ((int64_t(1) << nwin_bits) < (nrows + win - 1) / win) ++nwin_bits;
        const int end_bit = 32 + nwin_bits;
        size_t tmp_bytes = 0;
        DCHK(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, keys, keys_out, rows, slot_row, int(nrows), 0,
                                                end_bit, s));
        void *tmp = nullptr;
        DCHK(T.alloc(&tmp, tmp_bytes));
        DCHK(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, keys, keys_out, rows, slot_row, int(nrows), 0,
                                                end_bit, s));
    }
    if (sort) {
        hipLaunchKernelGGL(perm_tail_kernel, dim3(grid_for(nslots)), dim3(kT), 0, s, slot_row, nrows, nslots, flags);
        DCHK(hipGetLastError());
    }
    DCHK(hipMemcpyAsync(hflags, flags, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DCHK(hipStreamSynchronize(s));
    if (hflags[0] || hflags[1]) return SELL_ERR_ARG;
    const bool has_perm = sort && hflags[2];
    if (sort && !has_perm) {  // the sort kept every row in place: no permutation
        DCHK(lib_free(slot_row));
        M->d_perm = nullptr;
        slot_row = nullptr;
    }

    // chunk lengths and starts
    DCHK(lib_malloc(reinterpret_cast<void **>(&M->d_cl), sizeof(int32_t) * size_t(std::max<int64_t>(nch, 1))));
    DCHK(lib_malloc(reinterpret_cast<void **>(&M->d_cs), sizeof(int64_t) * (size_t(nch) + 1)));
    DCHK(T.alloc(reinterpret_cast<void **>(&csz), sizeof(int64_t) * (size_t(nch) + 1)));
    hipLaunchKernelGGL(chunk_len_kernel, dim3(grid_for(nch + 1)), dim3(kT), 0, s, len, slot_row, nrows, nch, C,
                       M->d_cl, csz);
    DCHK(hipGetLastError());
    {
        size_t tmp_bytes = 0;
        DCHK(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, csz, M->d_cs, int(nch + 1), s));
        void *tmp = nullptr;
        DCHK(T.alloc(&tmp, tmp_bytes));
        DCHK(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, csz, M->d_cs, int(nch + 1), s));
    }
    h.cl.resize(size_t(nch));
    h.cs.resize(size_t(nch) + 1);
    if (nch > 0) DCHK(hipMemcpyAsync(h.cl.data(), M->d_cl, sizeof(int32_t) * size_t(nch), hipMemcpyDeviceToHost, s));
    DCHK(hipMemcpyAsync(h.cs.data(), M->d_cs, sizeof(int64_t) * (size_t(nch) + 1), hipMemcpyDeviceToHost, s));
    DCHK(hipStreamSynchronize(s));
    const int64_t stored = h.cs[size_t(nch)];

    // the fill
    const int vb = dtype_bytes(vdt);
    DCHK(lib_malloc(reinterpret_cast<void **>(&M->d_col), sizeof(int32_t) * size_t(std::max<int64_t>(stored, 1))));
    DCHK(lib_malloc(&M->d_val, size_t(vb) * size_t(std::max<int64_t>(stored, 1))));
    if (nslots > 0) {
        if (vdt == SELL_F64)
            hipLaunchKernelGGL(fill_kernel<double>, dim3(grid_for(nslots)), dim3(kT), 0, s, rowptr, col, val, len,
                               slot_row, M->d_cl, M->d_cs, nrows, nslots, C, M->d_col,
                               static_cast<double *>(M->d_val));
        else if (vdt == SELL_F32)
            hipLaunchKernelGGL(fill_kernel<float>, dim3(grid_for(nslots)), dim3(kT), 0, s, rowptr, col, val, len,
                               slot_row, M->d_cl, M->d_cs, nrows, nslots, C, M->d_col, static_cast<float *>(M->d_val));
        else
            hipLaunchKernelGGL(fill_kernel<uint16_t>, dim3(grid_for(nslots)), dim3(kT), 0, s, rowptr, col, val, len,
                               slot_row, M->d_cl, M->d_cs, nrows, nslots, C, M->d_col,
                               static_cast<uint16_t *>(M->d_val));
        DCHK(hipGetLastError());
    }
    if (has_perm) {
        h.perm.resize(size_t(nslots));
        DCHK(hipMemcpyAsync(h.perm.data(), slot_row, sizeof(int32_t) * size_t(nslots), hipMemcpyDeviceToHost, s));
    }

    // the work partition, made on the host from the chunk lengths
    h.nrows = nrows;
    h.ncols = ncols;
    h.nnz = nnz;
    h.stored = stored;
    h.nch = nch;
    h.sigma = sigma;
    h.C = C;
    h.vdt = vdt;
    h.has_perm = has_perm;
    make_tiles(h.cl, C, default_tile_count(nch), h.tiles);
    h.batch = choose_batch_len(h.cl);
    h.batch_wide = choose_batch_len(h.cl, true);
    h.waves = choose_waves(h.cl);
    DCHK(lib_malloc(reinterpret_cast<void **>(&M->d_tiles), sizeof(int32_t) * h.tiles.size()));
    DCHK(hipMemcpyAsync(M->d_tiles, h.tiles.data(), sizeof(int32_t) * h.tiles.size(), hipMemcpyHostToDevice, s));
    DCHK(hipStreamSynchronize(s));
    M->ntiles = int32_t(h.tiles.size()) - 1;
    M->matrix_bytes = int64_t(stored) * (4 + vb) + nch * 12 + 8 + (has_perm ? nslots * 4 : 0) +
                      int64_t(h.tiles.size()) * 4;
    M->on_device = true;
    return SELL_OK;
#undef DCHK
}

}  // namespace sellcs
