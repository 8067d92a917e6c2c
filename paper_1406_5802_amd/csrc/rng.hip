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
//   Streams: 1 Gaussian G (element i*n+j = G[i][j]), 2 circulant c, 3 Toeplitz tau,
//   4 the phases of the unitary circulant (the uniforms themselves: element e
//   is u_{e mod 4} of block e / 4).
//
// Bound: HBM write of the output (8 or 4 bytes per element) plus ~300 VALU
// operations per block of four; one thread computes one block.
#include "bf16.h"
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

__global__ __launch_bounds__(256) void k_uniforms(double *__restrict__ out, int64_t count,
                                                  uint64_t seed, uint64_t stream) {
    const int64_t nblocks = (count + 3) / 4;
    const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t m = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; m < nblocks;
         m += step) {
        uint64_t w[4];
        Philox4x64::block(static_cast<uint64_t>(m), stream, seed, w);
        for (int j = 0; j < 4; ++j)
            if (4 * m + j < count) out[4 * m + j] = to_uniform(w[j]);
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

// The Gaussian multiplier of the split-BF16 path in one pass: each element
// drawn as above (stream `stream`, element i n + j), rounded FP64 -> FP32 ->
// BF16 (nearest, ties to even), and written both as its FP32 value into G
// (n x n) and, transposed, as BF16 bits into Ht (Ht[j][i] = H[i][j], row
// pitch ldk >= round_up(n, 64)).  64 x 64 tiles through LDS so both writes
// coalesce; n % 4 == 0, so each block of four lies in one row.
__global__ __launch_bounds__(256) void k_normals_bf16t(float *__restrict__ G,
                                                       uint16_t *__restrict__ Ht, int64_t n,
                                                       int64_t ldk, uint64_t seed,
                                                       uint64_t stream) {
    __shared__ uint16_t t[64][66];
    const int64_t i0 = static_cast<int64_t>(blockIdx.y) * 64, j0 = static_cast<int64_t>(blockIdx.x) * 64;
    const int tid = threadIdx.x, r = tid >> 4, cg = tid & 15;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        const int row = r + 16 * rr;
        const int64_t i = i0 + row, j = j0 + 4 * cg;
        uint16_t h[4] = {0, 0, 0, 0};
        if (i < n && j < n) {
            uint64_t w[4];
            Philox4x64::block(static_cast<uint64_t>((i * n + j) / 4), stream, seed, w);
            double z[4];
            box_muller(w, z);
            float v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                h[q] = bf16_bits(static_cast<float>(z[q]));
                v[q] = bf16_value(h[q]);
            }
            *reinterpret_cast<float4 *>(G + i * n + j) = float4{v[0], v[1], v[2], v[3]};
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) t[row][4 * cg + q] = h[q];
    }
    __syncthreads();
    const int jj = tid >> 2, ic = 8 * (tid & 3);
    const int64_t j = j0 + jj;
    if (j >= n) return;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        const int ib = ic + 32 * half;
        if (i0 + ib >= n) continue;  // rows past n: the padding keeps its zeros
        uint16_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = t[ib + u][jj];  // rows past n hold 0
        *reinterpret_cast<uint4 *>(Ht + j * ldk + i0 + ib) = pack8(v);
    }
}

// The multipliers of many systems in one launch.  Parameters of all systems
// form one index space of chunks of 1024 normals (256 blocks of four):
// chunk_start[s] is system s's first chunk (prefix sums, chunk_start[count]
// the total).  System s draws cnt[s] normals of stream stream[s] with seed
// seed[s], element e = output e mod 4 of block e / 4 as in k_normals: a dense
// Gaussian multiplier (stream 1, cnt = n^2) as FP32 values into g32 + off[s],
// a circulant's first column (stream 2, cnt = n) as FP64 into g64 + off[s].
__global__ __launch_bounds__(256) void k_batch_normals(
    int count, const int *__restrict__ chunk_start, const int64_t *__restrict__ cnt,
    const int *__restrict__ stream, const uint64_t *__restrict__ seed,
    const int64_t *__restrict__ off, float *g32, double *g64) {
    const int c = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {  // last s with chunk_start[s] <= c
        const int mid = (lo + hi + 1) >> 1;
        if (chunk_start[mid] <= c) lo = mid; else hi = mid - 1;
    }
    const int s = lo;
    const int64_t m = static_cast<int64_t>(c - chunk_start[s]) * 256 + threadIdx.x;
    const int64_t total = cnt[s];
    if (4 * m >= total) return;
    uint64_t w[4];
    Philox4x64::block(static_cast<uint64_t>(m), static_cast<uint64_t>(stream[s]), seed[s], w);
    double z[4];
    box_muller(w, z);
    for (int j = 0; j < 4; ++j) {
        const int64_t e = 4 * m + j;
        if (e >= total) break;
        if (stream[s] == 1)
            g32[off[s] + e] = static_cast<float>(z[j]);
        else
            g64[off[s] + e] = z[j];
    }
}

}  // namespace

hipError_t batch_normals(int count, int total_chunks, const int *chunk_start, const int64_t *cnt,
                         const int *stream, const uint64_t *seed, const int64_t *off, float *g32,
                         double *g64, hipStream_t s) {
    if (count <= 0 || total_chunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_normals, dim3(static_cast<unsigned>(total_chunks)), dim3(256), 0, s,
                       count, chunk_start, cnt, stream, seed, off, g32, g64);
    return hipGetLastError();
}

hipError_t launch_normals_f64(double *out, int64_t count, uint64_t seed, uint64_t stream,
                              hipStream_t s) {
    return launch_normals<double>(out, count, seed, stream, s);
}

hipError_t launch_uniforms_f64(double *out, int64_t count, uint64_t seed, uint64_t stream,
                               hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t grid = ((count + 3) / 4 + 255) / 256;
    if (grid > 256 * 64) grid = 256 * 64;
    hipLaunchKernelGGL(k_uniforms, dim3(static_cast<unsigned>(grid)), dim3(256), 0, s, out, count,
                       seed, stream);
    return hipGetLastError();
}

hipError_t launch_normals_f32(float *out, int64_t count, uint64_t seed, uint64_t stream,
                              hipStream_t s) {
    return launch_normals<float>(out, count, seed, stream, s);
}

hipError_t normals_bf16t(float *G, uint16_t *Ht, int64_t n, int64_t ldk, uint64_t seed,
                         uint64_t stream, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + 63) / 64;
    if (n % 4 != 0 || ldk % 8 != 0 || ldk < nb * 64 || nb > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_normals_bf16t, dim3(static_cast<unsigned>(nb), static_cast<unsigned>(nb)),
                       dim3(256), 0, s, G, Ht, n, ldk, seed, stream);
    return hipGetLastError();
}

}  // namespace rmge
