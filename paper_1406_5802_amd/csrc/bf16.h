// BF16 (1 sign, 8 exponent, 7 mantissa bits) conversions used by the
// split-BF16 kernels: rounding from FP32 to nearest, ties to even (NaN stays
// NaN), the value of a BF16 bit pattern, and packing eight patterns into one
// 16-byte word (element 0 in the low half of the first 32-bit lane).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace rmge {

__device__ inline uint16_t bf16_bits(float x) {
    const uint32_t b = __float_as_uint(x);
    if ((b & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((b >> 16) | 0x40u);
    return static_cast<uint16_t>((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}

__device__ inline float bf16_value(uint16_t h) {
    return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

__device__ inline uint4 pack8(const uint16_t *v) {
    return uint4{v[0] | (static_cast<uint32_t>(v[1]) << 16),
                 v[2] | (static_cast<uint32_t>(v[3]) << 16),
                 v[4] | (static_cast<uint32_t>(v[5]) << 16),
                 v[6] | (static_cast<uint32_t>(v[7]) << 16)};
}

}  // namespace rmge
