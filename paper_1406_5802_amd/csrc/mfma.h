// Wrappers of the two 16 x 16 x 4 matrix-core instructions used by the
// library (v_mfma_f64_16x16x4_f64 and v_mfma_f32_16x16x4_f32).
//
// Operand layouts, identical for both: lane l holds A[l & 15][l >> 4] of the
// 16 x 4 A block and B[l >> 4][l & 15] of the 4 x 16 B block.  Result: lane l,
// item r holds D[row(l, r)][l & 15] with row = (l >> 4) + 4 r for f64 and
// 4 (l >> 4) + r for f32 (measured on gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace rmge {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T>
struct Mma;

template <>
struct Mma<double> {
    using acc = v4d;
    __device__ static acc step(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <>
struct Mma<float> {
    using acc = v4f;
    __device__ static acc step(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

}  // namespace rmge
