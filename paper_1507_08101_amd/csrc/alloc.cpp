// alloc.cpp -- the library's device and pinned host allocations. Every one goes through these
// wrappers, which count the live allocations and can be told to fail the k-th next allocation
// with out-of-memory, so that tests can drive every error path of every entry point and check
// that nothing is left allocated.
#include <atomic>

#include "internal.h"

namespace sellcs {

namespace {

std::atomic<int64_t> g_fail_at{0};  // allocations until a forced failure (0: none)
std::atomic<int64_t> g_live{0};     // live allocations made through the wrappers

bool forced_failure() {
    int64_t k = g_fail_at.load();
    while (k > 0)
        if (g_fail_at.compare_exchange_weak(k, k - 1)) return k == 1;
    return false;
}

hipError_t counted(hipError_t e) {
    if (e == hipSuccess) g_live.fetch_add(1);
    return e;
}

}  // namespace

hipError_t lib_malloc(void **p, size_t bytes) {
    if (forced_failure()) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return counted(hipMalloc(p, bytes));
}

hipError_t lib_malloc_async(void **p, size_t bytes, hipStream_t s) {
    if (forced_failure()) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return counted(hipMallocAsync(p, bytes, s));
}

hipError_t lib_host_malloc(void **p, size_t bytes, unsigned flags) {
    if (forced_failure()) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return counted(hipHostMalloc(p, bytes, flags));
}

hipError_t lib_free(void *p) {
    if (!p) return hipSuccess;
    g_live.fetch_sub(1);
    return hipFree(p);
}

hipError_t lib_free_async(void *p, hipStream_t s) {
    if (!p) return hipSuccess;
    g_live.fetch_sub(1);
    return hipFreeAsync(p, s);
}

hipError_t lib_host_free(void *p) {
    if (!p) return hipSuccess;
    g_live.fetch_sub(1);
    return hipHostFree(p);
}

}  // namespace sellcs

extern "C" {

int sell_debug_fail_alloc(int64_t k) {
    if (k < 0) return SELL_ERR_ARG;
    sellcs::g_fail_at.store(k);
    return SELL_OK;
}

int sell_debug_live_allocs(int64_t *count) {
    if (!count) return SELL_ERR_ARG;
    *count = sellcs::g_live.load();
    return SELL_OK;
}

}  // extern "C"
