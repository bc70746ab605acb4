// devutil.h -- small device helpers shared by the kernels of libsellcs.
#pragma once

#include <hip/hip_runtime.h>

namespace sellcs {

// Sum of one value per thread of a 256-thread workgroup in a fixed order: butterfly inside
// each wave, then the four wave sums in order. The result is valid in thread 0.
__device__ __forceinline__ double block_sum_256(double v) {
    __shared__ double ws[4];
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) t = ((ws[0] + ws[1]) + ws[2]) + ws[3];
    __syncthreads();
    return t;
}

}  // namespace sellcs
