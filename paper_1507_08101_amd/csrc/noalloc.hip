// noalloc.hip -- sell_spmmv_aug_noalloc: the augmented product (same kernels as sell_spmmv_aug)
// with its reduction partials and lane scratch in a fixed device array instead of the per-stream
// workspace that sell_spmmv_aug allocates on its first call on a stream. For callers that cannot
// allocate device memory: code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc.
//
// The array is one per device (each device holds its own copy at its own address, found with
// hipGetSymbolAddress on the first call on that device) and lives until the process ends. Every
// call on a device shares it: calls that overlap on one device (different streams, or threads
// without ordering) race on the dot partials. Nothing in it needs to start at zero: every
// workgroup of a launch writes all of its partials before the finishing kernel, ordered after
// it on the same stream, reads them, and the lane scratch is only ever written.
#include <mutex>

#include "internal.h"

namespace {

using namespace sellcs;

// dot partials of one launch: at most kMaxTiles workgroups x 3 dots x kMaxSliceCols columns
constexpr size_t kNoAllocPartialBytes = size_t(kMaxTiles) * 3 * kMaxSliceCols * sizeof(double);
constexpr size_t kNoAllocBytes = kNoAllocPartialBytes + kScratchBytes;  // 6,324,224 bytes
static_assert(kNoAllocPartialBytes % 256 == 0, "lane scratch must stay 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char *g_ptr[kMaxDevices] = {};  // device address of the array, per device

// The array's device address on the current device (looked up once per device). In host code
// the name of the array is only a host-side stand-in: its address must never reach a kernel.
int scratch_address(unsigned char **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SELL_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return SELL_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return SELL_ERR_HIP;
        g_ptr[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_ptr[dev];
    return SELL_OK;
}

}  // namespace

extern "C" {

int sell_spmmv_aug_noalloc(const sell_mat *A, const sell_bv *X, sell_bv *Y, sell_bv *Z,
                           const sell_spmv_opts *opts, void *stream) {
    sell_spmv_opts o;
    int rc = check_aug_call(A, X, Y, Z, opts, &o);
    if (rc) return rc;
    // one launch writes 3 * (slice columns) * (workgroups) partials; workgroups never exceed the
    // matrix's tiles and slices never exceed kMaxSliceCols columns
    if (A->ntiles > kMaxTiles) return SELL_ERR_UNSUPPORTED;
    unsigned char *base = nullptr;
    if ((rc = scratch_address(&base))) return rc;
    Workspace ws;
    ws.partials = reinterpret_cast<double *>(base);
    ws.scratch = base + kNoAllocPartialBytes;
    const bool plain = (o.flags == 0);
    return aug_impl(A, X, Y, Z, o, !plain, static_cast<hipStream_t>(stream), nullptr, nullptr, &ws);
}

}  // extern "C"
