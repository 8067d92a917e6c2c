// Multiplier parameters: standard Gaussian variables (Definition defrndm:
// i.i.d., mean 0, variance 1) from a counter-based generator, so that any
// element can be drawn by any thread with no shared state.
//
// Generator: Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11).
//   key = (seed, 0), counter = (m, stream, 0, 0) for block m;
//   each block gives four 64-bit words w_0..w_3 and four uniforms
//   u_j = ((w_j >> 12) + 0.5) * 2^-52 (exact in binary64, strictly in (0, 1));
//   Box-Muller on (u_0, u_1) and (u_2, u_3):
//   z_0 = sqrt(-2 ln u_0) cos(2 pi u_1), z_1 = sqrt(-2 ln u_0) sin(2 pi u_1),
//   z_2, z_3 likewise; element e of a stream is z_{e mod 4} of block e / 4.
//   Streams: 1 Gaussian G (element i*n+j = G[i][j]), 2 circulant c, 3 Toeplitz tau.
//
// Bound: HBM write of the output (8 or 4 bytes per element) plus ~300 VALU
// operations per block of four; one thread computes one block.
#include "rmge_impl.h"

namespace rmge {
namespace {

struct Philox4x64 {
    static constexpr uint64_t kMul0 = 0xD2E7470EE14C6C93ull;
    static constexpr uint64_t kMul1 = 0xCA5A826395121157ull;
    static constexpr uint64_t kWeyl0 = 0x9E3779B97F4A7C15ull;
    static constexpr uint64_t kWeyl1 = 0xBB67AE8584CAA73Bull;

    __device__ static void block(uint64_t m, uint64_t stream, uint64_t seed, uint64_t w[4]) {
        uint64_t x0 = m, x1 = stream, x2 = 0, x3 = 0;
        uint64_t k0 = seed, k1 = 0;
#pragma unroll
        for (int r = 0; r < 10; ++r) {
            const uint64_t lo0 = kMul0 * x0, hi0 = __umul64hi(kMul0, x0);
            const uint64_t lo1 = kMul1 * x2, hi1 = __umul64hi(kMul1, x2);
            const uint64_t y0 = hi1 ^ x1 ^ k0;
            const uint64_t y2 = hi0 ^ x3 ^ k1;
            x0 = y0;
            x1 = lo1;
            x2 = y2;
            x3 = lo0;
            k0 += kWeyl0;
            k1 += kWeyl1;
        }
        w[0] = x0;
        w[1] = x1;
        w[2] = x2;
        w[3] = x3;
    }
};

__device__ inline double to_uniform(uint64_t w) {
    return (static_cast<double>(w >> 12) + 0.5) * 0x1.0p-52;
}

__device__ inline void box_muller(const uint64_t w[4], double z[4]) {
#pragma clang fp contract(off)
    const double two_pi = 6.283185307179586476925286766559;
    const double u0 = to_uniform(w[0]), u1 = to_uniform(w[1]);
    const double u2 = to_uniform(w[2]), u3 = to_uniform(w[3]);
    const double r01 = sqrt(-2.0 * log(u0));
    const double r23 = sqrt(-2.0 * log(u2));
    z[0] = r01 * cos(two_pi * u1);
    z[1] = r01 * sin(two_pi * u1);
    z[2] = r23 * cos(two_pi * u3);
    z[3] = r23 * sin(two_pi * u3);
}

template <typename T>
__global__ __launch_bounds__(256) void k_normals(T *__restrict__ out, int64_t count, uint64_t seed,
                                                 uint64_t stream) {
    const int64_t nblocks = (count + 3) / 4;
    const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t m = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; m < nblocks;
         m += step) {
        uint64_t w[4];
        Philox4x64::block(static_cast<uint64_t>(m), stream, seed, w);
        double z[4];
        box_muller(w, z);
        const int64_t e = 4 * m;
        if (e + 3 < count) {
#pragma unroll
            for (int j = 0; j < 4; ++j) out[e + j] = static_cast<T>(z[j]);
        } else {
            for (int j = 0; j < 4; ++j)
                if (e + j < count) out[e + j] = static_cast<T>(z[j]);
        }
    }
}

template <typename T>
hipError_t launch_normals(T *out, int64_t count, uint64_t seed, uint64_t stream, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int64_t nblocks = (count + 3) / 4;
    const int threads = 256;
    int64_t grid = (nblocks + threads - 1) / threads;
    if (grid > 256 * 64) grid = 256 * 64;  // grid-stride beyond 64 waves per CU
    hipLaunchKernelGGL(k_normals<T>, dim3(static_cast<unsigned>(grid)), dim3(threads), 0, s, out,
                       count, seed, stream);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_normals_f64(double *out, int64_t count, uint64_t seed, uint64_t stream,
                              hipStream_t s) {
    return launch_normals<double>(out, count, seed, stream, s);
}

hipError_t launch_normals_f32(float *out, int64_t count, uint64_t seed, uint64_t stream,
                              hipStream_t s) {
    return launch_normals<float>(out, count, seed, stream, s);
}

}  // namespace rmge
