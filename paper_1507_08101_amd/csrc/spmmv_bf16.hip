// spmmv_bf16.hip -- instantiations of the product kernels for one value/vector type pair.
#include "spmmv_impl.h"

namespace sellcs {

int prod_bf16(ProdArgs &a, bool aug, bool fixed_ok, hipStream_t s) {
    return aug ? dispatch_prod<VK_BF16F32, true>(a, s, fixed_ok) : dispatch_prod<VK_BF16F32, false>(a, s, fixed_ok);
}

int transpose_bf16(ProdArgs &a, hipStream_t s) { return dispatch_transpose<VK_BF16F32>(a, s); }

}  // namespace sellcs
