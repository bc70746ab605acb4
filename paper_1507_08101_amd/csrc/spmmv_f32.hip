// spmmv_f32.hip -- instantiations of the product kernels for one value/vector type pair.
#include "spmmv_impl.h"

namespace sellcs {

int prod_f32(ProdArgs &a, bool aug, bool fixed_ok, hipStream_t s) {
    return aug ? dispatch_prod<VK_F32F32, true>(a, s, fixed_ok) : dispatch_prod<VK_F32F32, false>(a, s, fixed_ok);
}

int transpose_f32(ProdArgs &a, hipStream_t s) { return dispatch_transpose<VK_F32F32>(a, s); }

const void *batch_kernel_f32(int b, int vpt, bool aug, bool fixed_ok, int ub, int ubw, uint32_t flags) {
    return aug ? batch_kernel_for<VK_F32F32, true>(b, vpt, fixed_ok, ub, ubw, flags)
               : batch_kernel_for<VK_F32F32, false>(b, vpt, fixed_ok, ub, ubw, 0);
}

const void *batch_mixed_kernel_f32(bool aug) {
    return aug ? batch_mixed_kernel_for<VK_F32F32, true>() : batch_mixed_kernel_for<VK_F32F32, false>();
}

}  // namespace sellcs
