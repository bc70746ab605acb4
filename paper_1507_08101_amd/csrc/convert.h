// convert.h -- element conversions of the library (host and device).
// Narrowing conversions round to nearest, ties to even, directly from the source value.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sellcs {

__host__ __device__ inline uint64_t f64_bits(double v) {
    uint64_t u;
    __builtin_memcpy(&u, &v, 8);
    return u;
}

__host__ __device__ inline uint32_t f32_bits(float v) {
    uint32_t u;
    __builtin_memcpy(&u, &v, 4);
    return u;
}

__host__ __device__ inline float f32_from_bits(uint32_t u) {
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

// double -> bfloat16 bits (8 significant bits, binary32 exponent range).
__host__ __device__ inline uint16_t bf16_from_f64(double v) {
    const uint64_t u = f64_bits(v);
    const uint16_t sign = uint16_t((u >> 48) & 0x8000u);
    const uint64_t mag = u & 0x7FFFFFFFFFFFFFFFull;
    if (mag > 0x7FF0000000000000ull) return uint16_t(sign | 0x7FC0u);  // NaN -> quiet NaN
    if (mag == 0x7FF0000000000000ull) return uint16_t(sign | 0x7F80u); // infinity
    const int e = int(mag >> 52) - 1023;
    if (e >= -126) {
        // normal range: keep 7 of the 52 fraction bits, round away the other 45
        const uint64_t frac = mag & ((1ull << 52) - 1);
        uint64_t keep = frac >> 45;
        const uint64_t rest = frac & ((1ull << 45) - 1);
        const uint64_t half = 1ull << 44;
        if (rest > half || (rest == half && (keep & 1u))) keep += 1;
        int eb = e + 127;
        if (keep == 128) {
            keep = 0;
            eb += 1;
        }
        if (eb >= 255) return uint16_t(sign | 0x7F80u);  // overflow to infinity
        return uint16_t(sign | (uint16_t(eb) << 7) | uint16_t(keep));
    }
    // below the smallest normal: multiples of 2^-133; scaling by 2^133 is exact
    const double a = (v < 0 ? -v : v) * 0x1p133;  // in [0, 128)
    uint64_t r = uint64_t(a);
    const double fr = a - double(r);
    if (fr > 0.5 || (fr == 0.5 && (r & 1u))) r += 1;  // r == 128 is the smallest normal
    return uint16_t(sign | uint16_t(r));
}

// float -> bfloat16 bits.
__host__ __device__ inline uint16_t bf16_from_f32(float v) {
    const uint32_t u = f32_bits(v);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return uint16_t(((u >> 16) & 0x8000u) | 0x7FC0u);
    const uint32_t lsb = (u >> 16) & 1u;
    return uint16_t((u + 0x7FFFu + lsb) >> 16);
}

__host__ __device__ inline float f32_from_bf16(uint16_t b) { return f32_from_bits(uint32_t(b) << 16); }

// Generic element conversion used by the block-vector copy.
template <class D, class S>
struct Conv;
template <>
struct Conv<double, double> {
    __host__ __device__ static double go(double v) { return v; }
};
template <>
struct Conv<float, double> {
    __host__ __device__ static float go(double v) { return float(v); }
};
template <>
struct Conv<uint16_t, double> {
    __host__ __device__ static uint16_t go(double v) { return bf16_from_f64(v); }
};
template <>
struct Conv<double, float> {
    __host__ __device__ static double go(float v) { return double(v); }
};
template <>
struct Conv<float, float> {
    __host__ __device__ static float go(float v) { return v; }
};
template <>
struct Conv<uint16_t, float> {
    __host__ __device__ static uint16_t go(float v) { return bf16_from_f32(v); }
};
template <>
struct Conv<double, uint16_t> {
    __host__ __device__ static double go(uint16_t v) { return double(f32_from_bf16(v)); }
};
template <>
struct Conv<float, uint16_t> {
    __host__ __device__ static float go(uint16_t v) { return f32_from_bf16(v); }
};
template <>
struct Conv<uint16_t, uint16_t> {
    __host__ __device__ static uint16_t go(uint16_t v) { return v; }
};

}  // namespace sellcs
