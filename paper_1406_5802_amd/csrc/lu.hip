// Pivot blocks of block Gaussian elimination with no pivoting.
//
// Section 3 of the paper factors A = [[B, C], [D, E]] as in eq. eqgenp and
// recurses on the pivot block B and on the Schur complement S = E - D B^{-1} C;
// with pivot blocks of size 1 this is GENP, and by the order-independence
// argument after eq. eqgenpin every choice of block sizes produces the same
// Schur complements.  The host driver (api.hip) walks the matrix in panels of
// `block` columns.  This file holds
//   * k_leaf_lu: one pivot block of at most 128 x 128 factored entirely in LDS
//     by one workgroup, pivot by pivot, plus the inverses of the 32 x 32
//     diagonal sub-blocks of its two triangular factors;
//   * k_trsm: B^{-1} C = U_B^{-1} (L_B^{-1} C) and D B^{-1} = (D U_B^{-1}) L_B^{-1}
//     split into the two triangular solves, each done in place by blocked
//     substitution on a strip staged in LDS: the 32 x 32 diagonal sub-blocks
//     are applied through their inverses, the rest as plain updates.  Only
//     small blocks are inverted, so the error grows with the condition of
//     32 x 32 blocks, not of the whole pivot block.
//
// Breakdown: a pivot that is exactly 0 (Corollary corec: the input is not
// strongly nonsingular) or not finite stops the elimination; its global index
// is recorded in the device status word and every later kernel exits early.
//
// Bound: the leaf is latency bound (b sequential pivot steps, two barriers
// each); the solves issue one LDS read per multiply-add (VALU/LDS bound) and
// carry b^2 / 2 multiply-adds per strip column.
#include "rmge_impl.h"

namespace rmge {
namespace {

constexpr int kLd = kLeaf + 1;  // LDS row stride (one element of padding)
constexpr int kSub = 32;        // diagonal sub-blocks that are inverted explicitly
constexpr int kInvLdDev = kMaxBlock;

template <typename T>
__device__ inline bool is_bad(T p) {
    return p == T(0) || !isfinite(p);
}

template <typename T>
__global__ __launch_bounds__(1024) void k_leaf_lu(T *a, int64_t lda, int b, T *Linv, T *Uinv,
                                                  int64_t ldw, int64_t k0, DevStatus *st) {
    __shared__ T s[kLeaf * kLd];
    __shared__ T red[4][8][kSub];
    if (st->code != 0) return;  // an earlier pivot block broke down
    const int tid = threadIdx.x;
    const int tx = tid & 31, ty = tid >> 5;  // 32 x 32 thread grid

    for (int i = ty; i < b; i += 32)
        for (int j = tx; j < b; j += 32) s[i * kLd + j] = a[static_cast<int64_t>(i) * lda + j];
    __syncthreads();

    // Unblocked elimination, pivot by pivot (eq. eqgenp with 1 x 1 pivot blocks).
    int done = b;
    for (int j = 0; j < b; ++j) {
        const T p = s[j * kLd + j];
        if (is_bad(p)) {
            if (tid == 0) {
                st->info = k0 + j;
                st->code = (p == T(0)) ? 4 : 5;
            }
            done = j;
            break;
        }
        for (int i = j + 1 + tid; i < b; i += 1024) s[i * kLd + j] = s[i * kLd + j] / p;
        __syncthreads();
        for (int i = j + 1 + ty; i < b; i += 32) {
            const T l = s[i * kLd + j];
            for (int c = j + 1 + tx; c < b; c += 32) s[i * kLd + c] -= l * s[j * kLd + c];
        }
        __syncthreads();
    }

    for (int i = ty; i < b; i += 32)
        for (int j = tx; j < b; j += 32) a[static_cast<int64_t>(i) * lda + j] = s[i * kLd + j];
    if (done < b) return;

    // Inverses of the 32 x 32 diagonal sub-blocks of U and of the unit lower
    // factor, in place in LDS; the off-diagonal coupling is applied later by
    // blocked substitution (k_trsm), so only these small inverses are formed.
    // Threads: 4 sub-blocks x 32 columns x 8 partial sums.
    const int q = tid >> 8, col = tid & 31, part = (tid >> 5) & 7;
    const int q0 = q * kSub;
    const int sbq = (b - q0) < kSub ? (b - q0) : kSub;  // may be <= 0 for small b
    // U_qq^{-1}, bottom row first: X[i][i] = 1/U[i][i], X[i][c] = -X[i][i] sum_{k=i+1..c} U[i][k] X[k][c].
    for (int i = kSub - 1; i >= 0; --i) {
        const bool act = i < sbq;
        T acc = T(0);
        if (act && col > i && col < sbq)
            for (int k = i + 1 + part; k <= col; k += 8)
                acc += s[(q0 + i) * kLd + q0 + k] * s[(q0 + k) * kLd + q0 + col];
        red[q][part][col] = acc;
        const T d = act ? T(1) / s[(q0 + i) * kLd + q0 + i] : T(0);  // read before row i changes
        __syncthreads();
        if (act && part == 0 && col >= i && col < sbq) {
            if (col == i) {
                s[(q0 + i) * kLd + q0 + i] = d;
            } else {
                T sum = T(0);
#pragma unroll
                for (int r = 0; r < 8; ++r) sum += red[q][r][col];
                s[(q0 + i) * kLd + q0 + col] = -d * sum;
            }
        }
        __syncthreads();
    }
    // L_qq^{-1} (unit diagonal), top row first: X[i][c] = -(L[i][c] + sum_{k=c+1..i-1} L[i][k] X[k][c]).
    for (int i = 1; i < kSub; ++i) {
        const bool act = i < sbq;
        T acc = T(0);
        if (act && col < i)
            for (int k = col + 1 + part; k < i; k += 8)
                acc += s[(q0 + i) * kLd + q0 + k] * s[(q0 + k) * kLd + q0 + col];
        red[q][part][col] = acc;
        __syncthreads();
        if (act && part == 0 && col < i) {
            T sum = s[(q0 + i) * kLd + q0 + col];
#pragma unroll
            for (int r = 0; r < 8; ++r) sum += red[q][r][col];
            s[(q0 + i) * kLd + q0 + col] = -sum;
        }
        __syncthreads();
    }
    if (sbq > 0 && part < 4) {
        for (int i = part; i < sbq; i += 4) {
            if (col >= sbq) continue;
            const T v = s[(q0 + i) * kLd + q0 + col];
            const int64_t o = static_cast<int64_t>(q0 + i) * ldw + q0 + col;
            Uinv[o] = (col >= i) ? v : T(0);
            Linv[o] = (col < i) ? v : (col == i ? T(1) : T(0));
        }
    }
}

// Blocked substitution with the packed pivot block of width b (<= 256) at
// `lu` (ld), in place on a strip of the panel, using the inverses of the
// 32 x 32 diagonal sub-blocks (Linv / Uinv, ld kInvLd):
//   LEFT  (kind 0): X = L^{-1} C   for a 256-row x 32-column strip of C = A12;
//   RIGHT (kind 1): X = D U^{-1}   for a 32-row x 256-column strip of D = A21,
//                   done as the left solve X^T = U^{-T} D^T on the transposed strip.
// The strip and the current sub-block column of the factor are staged in LDS;
// thread (c, g) owns column c of the (transposed) strip and rows g, g + 8, ...
template <typename T, int SIDE>
__global__ __launch_bounds__(256) void k_trsm(const T *lu, int64_t ld, int b, T *C, int64_t ldc,
                                              int64_t count, const T *Dinv, const int *abort) {
    constexpr int W = 32, LS = W + 1;
    __shared__ T S[kMaxBlock * LS];      // strip, S[k][c]
    __shared__ T P[(kMaxBlock - kSub) * LS];  // factor rows below the current sub-block
    __shared__ T Dv[kSub * LS];          // current diagonal sub-block inverse
    if (abort != nullptr && *abort != 0) return;
    const int tid = threadIdx.x, c = tid & (W - 1), g = tid >> 5;
    const int64_t c0 = static_cast<int64_t>(blockIdx.x) * W;
    const int w = static_cast<int>((count - c0) < W ? (count - c0) : W);
    // load the strip
    if (SIDE == 0) {
        for (int e = tid; e < b * W; e += 256) {
            const int k = e / W, cc = e % W;
            S[k * LS + cc] = cc < w ? C[k * ldc + c0 + cc] : T(0);
        }
    } else {
        for (int e = tid; e < b * W; e += 256) {
            const int cc = e / b, k = e % b;
            S[k * LS + cc] = cc < w ? C[(c0 + cc) * ldc + k] : T(0);
        }
    }
    for (int i0 = 0; i0 < b; i0 += kSub) {
        const int sb = (b - i0) < kSub ? (b - i0) : kSub;
        const int e0 = i0 + sb, below = b - e0;
        // stage the diagonal inverse (transposed for the right side) and the coupling panel
        for (int e = tid; e < sb * sb; e += 256) {
            const int r = e / sb, k = e % sb;
            Dv[r * LS + k] = (SIDE == 0) ? Dinv[(i0 + r) * static_cast<int64_t>(kInvLdDev) + i0 + k]
                                         : Dinv[(i0 + k) * static_cast<int64_t>(kInvLdDev) + i0 + r];
        }
        if (SIDE == 0) {
            for (int e = tid; e < below * sb; e += 256) {
                const int r = e / sb, k = e % sb;
                P[r * LS + k] = lu[(e0 + r) * ld + i0 + k];
            }
        } else {
            for (int e = tid; e < below * sb; e += 256) {
                const int k = e / below, r = e % below;
                P[r * LS + k] = lu[(i0 + k) * ld + e0 + r];
            }
        }
        __syncthreads();
        // X_i = Dinv_i S_i
        T x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r = g + 8 * u;
            T acc = T(0);
            if (r < sb)
                for (int k = 0; k < sb; ++k) acc += Dv[r * LS + k] * S[(i0 + k) * LS + c];
            x[u] = acc;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r = g + 8 * u;
            if (r < sb) S[(i0 + r) * LS + c] = x[u];
        }
        __syncthreads();
        // rows below: S_r -= P_r X_i
        for (int r = g; r < below; r += 8) {
            T acc = T(0);
            for (int k = 0; k < sb; ++k) acc += P[r * LS + k] * S[(i0 + k) * LS + c];
            S[(e0 + r) * LS + c] -= acc;
        }
        __syncthreads();
    }
    if (SIDE == 0) {
        for (int e = tid; e < b * W; e += 256) {
            const int k = e / W, cc = e % W;
            if (cc < w) C[k * ldc + c0 + cc] = S[k * LS + cc];
        }
    } else {
        for (int e = tid; e < b * W; e += 256) {
            const int cc = e / b, k = e % b;
            if (cc < w) C[(c0 + cc) * ldc + k] = S[k * LS + cc];
        }
    }
}

template <typename T>
__global__ void k_set_identity(T *a, int64_t ld, int64_t n) {
    const int64_t total = n * n;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t i = e / n, j = e % n;
        a[i * ld + j] = (i == j) ? T(1) : T(0);
    }
}

template <typename T, typename U>
__global__ void k_convert_2d(const T *src, int64_t lds, U *dst, int64_t ldd, int64_t rows,
                             int64_t cols) {
    const int64_t total = rows * cols;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t i = e / cols, j = e % cols;
        dst[i * ldd + j] = static_cast<U>(src[i * lds + j]);
    }
}

__device__ inline void atomic_max_nonneg(double *addr, double v) {
    // Non-negative doubles order like their bit patterns (NaN sorts above Inf).
    atomicMax(reinterpret_cast<unsigned long long *>(addr),
              static_cast<unsigned long long>(__double_as_longlong(v)));
}

__device__ inline void atomic_min_nonneg(double *addr, double v) {
    atomicMin(reinterpret_cast<unsigned long long *>(addr),
              static_cast<unsigned long long>(__double_as_longlong(v)));
}

// out[0] = max |U| (upper triangle incl. diagonal), out[1] = min |u_kk|, out[2] = max |A|
// over the full n x n matrix (the latter only when `full` is set).
template <typename T>
__global__ void k_lu_stats(const T *lu, int64_t ld, int64_t n, double *out, int full) {
    double umax = 0.0, dmin = INFINITY, amax = 0.0;
    const int64_t total = n * n;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t i = e / n, j = e % n;
        const double v = fabs(static_cast<double>(lu[i * ld + j]));
        if (full) amax = fmax(amax, v);
        if (j >= i) umax = fmax(umax, v);
        if (j == i) dmin = fmin(dmin, v);
    }
    for (int off = 32; off > 0; off >>= 1) {
        umax = fmax(umax, __shfl_xor(umax, off));
        dmin = fmin(dmin, __shfl_xor(dmin, off));
        amax = fmax(amax, __shfl_xor(amax, off));
    }
    if ((threadIdx.x & 63) == 0) {
        if (full) {
            atomic_max_nonneg(out + 2, amax);
        } else {
            atomic_max_nonneg(out + 0, umax);
            atomic_min_nonneg(out + 1, dmin);
        }
    }
}

int grid_for(int64_t total, int threads) {
    int64_t g = (total + threads - 1) / threads;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return static_cast<int>(g);
}

}  // namespace

template <typename T>
hipError_t leaf_lu(T *a, int64_t lda, int b, T *Linv, T *Uinv, int64_t ldw, int64_t k0,
                   DevStatus *st, hipStream_t s) {
    if (b < 1 || b > kLeaf) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_leaf_lu<T>, dim3(1), dim3(1024), 0, s, a, lda, b, Linv, Uinv, ldw, k0, st);
    return hipGetLastError();
}

template <typename T>
hipError_t trsm(int side, const T *lu, int64_t ld, int b, T *C, int64_t ldc, int64_t count,
                const T *Dinv, const int *abort, hipStream_t s) {
    if (b < 1 || b > kMaxBlock) return hipErrorInvalidValue;
    if (count <= 0) return hipSuccess;
    const unsigned grid = static_cast<unsigned>((count + 31) / 32);
    if (side == 0)
        hipLaunchKernelGGL((k_trsm<T, 0>), dim3(grid), dim3(256), 0, s, lu, ld, b, C, ldc, count,
                           Dinv, abort);
    else
        hipLaunchKernelGGL((k_trsm<T, 1>), dim3(grid), dim3(256), 0, s, lu, ld, b, C, ldc, count,
                           Dinv, abort);
    return hipGetLastError();
}

template <typename T>
hipError_t set_identity(T *a, int64_t ld, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_set_identity<T>, dim3(grid_for(n * n, 256)), dim3(256), 0, s, a, ld, n);
    return hipGetLastError();
}

template <typename T, typename U>
hipError_t convert_2d(const T *src, int64_t lds, U *dst, int64_t ldd, int64_t rows, int64_t cols,
                      hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_convert_2d<T, U>), dim3(grid_for(rows * cols, 256)), dim3(256), 0, s,
                       src, lds, dst, ldd, rows, cols);
    return hipGetLastError();
}

// out3 must be preset to {0, +Inf, *} (max |U|, min |u_kk|); `full` variant writes out3[2].
template <typename T>
hipError_t lu_stats(const T *lu, int64_t ld, int64_t n, double *out3, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lu_stats<T>, dim3(grid_for(n * n, 256)), dim3(256), 0, s, lu, ld, n, out3,
                       0);
    return hipGetLastError();
}

template <typename T>
hipError_t abs_max(const T *m, int64_t ld, int64_t n, double *out3, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lu_stats<T>, dim3(grid_for(n * n, 256)), dim3(256), 0, s, m, ld, n, out3,
                       1);
    return hipGetLastError();
}

template hipError_t leaf_lu<double>(double *, int64_t, int, double *, double *, int64_t, int64_t,
                                    DevStatus *, hipStream_t);
template hipError_t leaf_lu<float>(float *, int64_t, int, float *, float *, int64_t, int64_t,
                                   DevStatus *, hipStream_t);
template hipError_t trsm<double>(int, const double *, int64_t, int, double *, int64_t, int64_t,
                                 const double *, const int *, hipStream_t);
template hipError_t trsm<float>(int, const float *, int64_t, int, float *, int64_t, int64_t,
                                const float *, const int *, hipStream_t);
template hipError_t set_identity<double>(double *, int64_t, int64_t, hipStream_t);
template hipError_t set_identity<float>(float *, int64_t, int64_t, hipStream_t);
template hipError_t convert_2d<double, double>(const double *, int64_t, double *, int64_t, int64_t,
                                               int64_t, hipStream_t);
template hipError_t convert_2d<double, float>(const double *, int64_t, float *, int64_t, int64_t,
                                              int64_t, hipStream_t);
template hipError_t convert_2d<float, double>(const float *, int64_t, double *, int64_t, int64_t,
                                              int64_t, hipStream_t);
template hipError_t convert_2d<float, float>(const float *, int64_t, float *, int64_t, int64_t,
                                             int64_t, hipStream_t);
template hipError_t lu_stats<double>(const double *, int64_t, int64_t, double *, hipStream_t);
template hipError_t lu_stats<float>(const float *, int64_t, int64_t, double *, hipStream_t);
template hipError_t abs_max<double>(const double *, int64_t, int64_t, double *, hipStream_t);
template hipError_t abs_max<float>(const float *, int64_t, int64_t, double *, hipStream_t);

}  // namespace rmge
