// Triangular solves, back-transformation and refinement residuals.
//
// After M = A H = L U, the solution of A x = b is x = H U^{-1} L^{-1} b
// (Fact faprepr), and its transpose gives the adjoint A^{-T} w =
// L^{-T} U^{-T} H^T w.  Refinement (Section 8.1) needs r = b - A x in FP64.
// Every kernel here streams a matrix once and is bound by HBM bandwidth.
//
// Triangular solves are blocked by 64 rows: each 64 x 64 diagonal block is
// solved in registers by one wave (lane = row, wavefront shuffles broadcast
// each solved value) and the coupling tiles are staged through LDS so that
// their global reads are row segments (coalesced) for plain and transposed
// factors alike.  k_trsv_persistent does a whole solve in one launch;
// k_trsv_step does one diagonal block per launch (kept for reference use).
#include "rmge_impl.h"

namespace rmge {
namespace {

constexpr int SB = 64;

template <typename T, int MODE, int NR>
__global__ __launch_bounds__(256) void k_trsv_step(const T *LU, int64_t ld, int64_t n, int64_t blk,
                                                   T *Y, T *X, int64_t ldyx, int nr,
                                                   const int *abort) {
    __shared__ T Ds[SB][SB + 1];
    __shared__ T Ts[SB][SB + 1];
    __shared__ T xs[SB][NR];
    if (abort != nullptr && *abort != 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t I0 = blk * SB;
    const int bI = static_cast<int>((n - I0) < SB ? (n - I0) : SB);

    for (int e = tid; e < SB * SB; e += 256) {
        const int i = e / SB, j = e % SB;
        Ds[i][j] = (i < bI && j < bI) ? LU[(I0 + i) * ld + I0 + j] : T(0);
    }
    __syncthreads();

    if (wave == 0) {
        T v[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r)
            v[r] = (lane < bI && r < nr) ? Y[(I0 + lane) * ldyx + r] : T(0);
        if (MODE == 0) {  // L: unit lower, forward
            for (int j = 0; j < bI; ++j) {
                const T l = Ds[lane][j];
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const T t = __shfl(v[r], j);
                    if (lane > j) v[r] -= l * t;
                }
            }
        } else if (MODE == 1) {  // U: upper, backward
            for (int j = bI - 1; j >= 0; --j) {
                const T d = Ds[j][j], u = Ds[lane][j];
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    if (lane == j) v[r] = v[r] / d;
                    const T t = __shfl(v[r], j);
                    if (lane < j) v[r] -= u * t;
                }
            }
        } else if (MODE == 2) {  // U^T: lower, forward
            for (int j = 0; j < bI; ++j) {
                const T d = Ds[j][j], u = Ds[j][lane];
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    if (lane == j) v[r] = v[r] / d;
                    const T t = __shfl(v[r], j);
                    if (lane > j) v[r] -= u * t;
                }
            }
        } else {  // L^T: unit upper, backward
            for (int j = bI - 1; j >= 0; --j) {
                const T l = Ds[j][lane];
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const T t = __shfl(v[r], j);
                    if (lane < j) v[r] -= l * t;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            xs[lane][r] = (lane < bI) ? v[r] : T(0);
            if (blockIdx.x == 0 && lane < bI && r < nr) X[(I0 + lane) * ldyx + r] = v[r];
        }
    }
    __syncthreads();

    const bool below = (MODE == 0 || MODE == 2);
    const int64_t R0 = below ? I0 + bI + static_cast<int64_t>(blockIdx.x) * SB
                             : static_cast<int64_t>(blockIdx.x) * SB;
    const int64_t rend = below ? n : I0;
    if (R0 >= rend) return;
    const int rows = static_cast<int>((rend - R0) < SB ? (rend - R0) : SB);
    if (MODE == 0 || MODE == 1) {
        for (int e = tid; e < SB * SB; e += 256) {
            const int r = e / SB, j = e % SB;
            Ts[r][j] = (r < rows && j < bI) ? LU[(R0 + r) * ld + I0 + j] : T(0);
        }
    } else {
        for (int e = tid; e < SB * SB; e += 256) {
            const int j = e / SB, r = e % SB;
            Ts[r][j] = (r < rows && j < bI) ? LU[(I0 + j) * ld + R0 + r] : T(0);
        }
    }
    __syncthreads();
    const int r = tid >> 2, q = tid & 3;
    if (r < rows) {
        for (int c = q; c < nr; c += 4) {
            T acc = T(0);
#pragma unroll 8
            for (int j = 0; j < SB; ++j) acc += Ts[r][j] * xs[j][c];
            Y[(R0 + r) * ldyx + c] -= acc;
        }
    }
}

// Whole triangular solve in one launch.  Workgroups take block rows in the
// order they start (a ticket from an atomic counter), so every block a
// workgroup waits on belongs to a workgroup that is already running; block I
// accumulates the coupling T_IJ y_J of every finished block J (waiting on
// J's flag), then solves its diagonal block and publishes y_I with a release
// fence and its flag.  A wait gives up after kSpinLimit polls and records an
// error instead of hanging; the caller checks it.
constexpr int kSpinLimit = 1 << 22;

template <typename T, int MODE, int NR>
__global__ __launch_bounds__(256) void k_trsv_persistent(const T *LU, int64_t ld, int64_t n,
                                                         const T *B, T *X, int64_t ldx, int nr,
                                                         int *counter, int *flags, int epoch,
                                                         int *err) {
    __shared__ T Ds[SB][SB + 1];  // diagonal block
    __shared__ T Ts[SB][SB + 1];  // coupling tile T_IJ
    __shared__ T ys[SB][NR];
    __shared__ int s_ticket, s_fail;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool forward = (MODE == 0 || MODE == 2);
    const bool transposed = (MODE == 2 || MODE == 3);
    if (tid == 0) {
        s_ticket = atomicAdd(counter, 1);
        s_fail = 0;
    }
    __syncthreads();
    const int nblk = static_cast<int>((n + SB - 1) / SB);
    const int I = forward ? s_ticket : nblk - 1 - s_ticket;
    const int64_t I0 = static_cast<int64_t>(I) * SB;
    const int bI = static_cast<int>((n - I0) < SB ? (n - I0) : SB);
    const int r = tid >> 2, q = tid & 3;  // row r of the block, column quarter q
    // Everything that does not depend on other blocks is loaded before waiting.
    for (int e = tid; e < SB * SB; e += 256) {
        const int i = e / SB, j = e % SB;
        Ds[i][j] = (i < bI && j < bI) ? LU[(I0 + i) * ld + I0 + j] : T(0);
    }
    T bval[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c)
        bval[c] = (q == 0 && r < bI && c < nr) ? B[(I0 + r) * ldx + c] : T(0);
    double acc[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = 0.0;
    const int jfirst = forward ? 0 : nblk - 1, jstep = forward ? 1 : -1;
    for (int J = jfirst; J != I; J += jstep) {
        const int64_t J0 = static_cast<int64_t>(J) * SB;
        const int bJ = static_cast<int>((n - J0) < SB ? (n - J0) : SB);
        // the coupling tile T_IJ (rows of this block, columns of block J)
        if (!transposed) {
            for (int e = tid; e < SB * SB; e += 256) {
                const int rr = e / SB, cc = e % SB;
                Ts[rr][cc] = (rr < bI && cc < bJ) ? LU[(I0 + rr) * ld + J0 + cc] : T(0);
            }
        } else {
            for (int e = tid; e < SB * SB; e += 256) {
                const int cc = e / SB, rr = e % SB;  // T[r][c] = factor[J0 + c][I0 + r]
                Ts[rr][cc] = (rr < bI && cc < bJ) ? LU[(J0 + cc) * ld + I0 + rr] : T(0);
            }
        }
        if (tid == 0) {
            int spins = 0;
            while (__hip_atomic_load(flags + J, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
                if (++spins > kSpinLimit ||
                    __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                    s_fail = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __syncthreads();
        if (s_fail) break;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        for (int e = tid; e < SB * NR; e += 256) {
            const int rr = e / NR, c = e % NR;
            ys[rr][c] = (rr < bJ && c < nr) ? X[(J0 + rr) * ldx + c] : T(0);
        }
        __syncthreads();
#pragma unroll 4
        for (int k = 16 * q; k < 16 * q + 16; ++k) {
            const double t = static_cast<double>(Ts[r][k]);
#pragma unroll
            for (int c = 0; c < NR; ++c) acc[c] += t * static_cast<double>(ys[k][c]);
        }
        __syncthreads();
    }
    if (s_fail) {
        if (tid == 0) atomicExch(err, 1);  // blocks waiting on this one see it and stop
        return;
    }
    // reduce the four column quarters of each row, form the right-hand side
#pragma unroll
    for (int c = 0; c < NR; ++c) {
        acc[c] += __shfl_xor(acc[c], 1);
        acc[c] += __shfl_xor(acc[c], 2);
    }
    if (q == 0) {
#pragma unroll
        for (int c = 0; c < NR; ++c)
            ys[r][c] = static_cast<T>(static_cast<double>(bval[c]) - acc[c]);
    }
    __syncthreads();
    if (wave == 0) {
        T v[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c) v[c] = ys[lane][c];
        if (MODE == 0) {
            for (int j = 0; j < bI; ++j) {
                const T l = Ds[lane][j];
#pragma unroll
                for (int c = 0; c < NR; ++c) {
                    const T t = __shfl(v[c], j);
                    if (lane > j) v[c] -= l * t;
                }
            }
        } else if (MODE == 1) {
            for (int j = bI - 1; j >= 0; --j) {
                const T d = Ds[j][j], u = Ds[lane][j];
#pragma unroll
                for (int c = 0; c < NR; ++c) {
                    if (lane == j) v[c] = v[c] / d;
                    const T t = __shfl(v[c], j);
                    if (lane < j) v[c] -= u * t;
                }
            }
        } else if (MODE == 2) {
            for (int j = 0; j < bI; ++j) {
                const T d = Ds[j][j], u = Ds[j][lane];
#pragma unroll
                for (int c = 0; c < NR; ++c) {
                    if (lane == j) v[c] = v[c] / d;
                    const T t = __shfl(v[c], j);
                    if (lane > j) v[c] -= u * t;
                }
            }
        } else {
            for (int j = bI - 1; j >= 0; --j) {
                const T l = Ds[j][lane];
#pragma unroll
                for (int c = 0; c < NR; ++c) {
                    const T t = __shfl(v[c], j);
                    if (lane < j) v[c] -= l * t;
                }
            }
        }
        if (lane < bI) {
#pragma unroll
            for (int c = 0; c < NR; ++c)
                if (c < nr) X[(I0 + lane) * ldx + c] = v[c];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (lane == 0) __hip_atomic_store(flags + I, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void k_trsv_reset(int *counter) { *counter = 0; }

template <typename T, int MODE>
hipError_t trsv_launch(const T *LU, int64_t ld, int64_t n, int64_t blk, T *Y, T *X, int64_t ldyx,
                       int nr, const int *abort, hipStream_t s) {
    const int64_t I0 = blk * SB;
    const int64_t bI = (n - I0) < SB ? (n - I0) : SB;
    const int64_t span = (MODE == 0 || MODE == 2) ? (n - I0 - bI) : I0;
    int64_t grid = (span + SB - 1) / SB;
    if (grid < 1) grid = 1;
    if (nr <= 1)
        hipLaunchKernelGGL((k_trsv_step<T, MODE, 1>), dim3(static_cast<unsigned>(grid)), dim3(256),
                           0, s, LU, ld, n, blk, Y, X, ldyx, nr, abort);
    else if (nr <= 4)
        hipLaunchKernelGGL((k_trsv_step<T, MODE, 4>), dim3(static_cast<unsigned>(grid)), dim3(256),
                           0, s, LU, ld, n, blk, Y, X, ldyx, nr, abort);
    else
        hipLaunchKernelGGL((k_trsv_step<T, MODE, 16>), dim3(static_cast<unsigned>(grid)), dim3(256),
                           0, s, LU, ld, n, blk, Y, X, ldyx, nr, abort);
    return hipGetLastError();
}

// y = beta y + alpha M x, FP64 accumulation; one wave per two rows.
template <typename TM, typename TX, typename TY, int NR>
__global__ __launch_bounds__(256) void k_gemv_n(int64_t rows, int64_t cols, double alpha,
                                                const TM *__restrict__ Mat, int64_t ldm,
                                                const TX *__restrict__ x, int64_t ldx, double beta,
                                                TY *y, int64_t ldy, int nrhs) {
    const int lane = threadIdx.x & 63;
    const int64_t row0 = (static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6)) * 2;
    if (row0 >= rows) return;
    const bool two = row0 + 1 < rows;
    double a0[NR], a1[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) a0[r] = a1[r] = 0.0;
    const TM *m0 = Mat + row0 * ldm;
    const TM *m1 = two ? m0 + ldm : m0;
    int64_t c = lane;
    for (; c + 192 < cols; c += 256) {
        double p0[4], p1[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            p0[u] = static_cast<double>(m0[c + 64 * u]);
            p1[u] = static_cast<double>(m1[c + 64 * u]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int r = 0; r < NR; ++r)
                if (r < nrhs) {
                    const double xv = static_cast<double>(x[(c + 64 * u) * ldx + r]);
                    a0[r] += p0[u] * xv;
                    a1[r] += p1[u] * xv;
                }
    }
    for (; c < cols; c += 64) {
        const double p0 = static_cast<double>(m0[c]), p1 = static_cast<double>(m1[c]);
#pragma unroll
        for (int r = 0; r < NR; ++r)
            if (r < nrhs) {
                const double xv = static_cast<double>(x[c * ldx + r]);
                a0[r] += p0 * xv;
                a1[r] += p1 * xv;
            }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        for (int off = 32; off > 0; off >>= 1) {
            a0[r] += __shfl_xor(a0[r], off);
            a1[r] += __shfl_xor(a1[r], off);
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
            if (r < nrhs) {
                TY *y0 = y + row0 * ldy + r;
                const double v0 = alpha * a0[r];
                *y0 = static_cast<TY>(beta == 0.0 ? v0 : v0 + beta * static_cast<double>(*y0));
                if (two) {
                    TY *y1 = y0 + ldy;
                    const double v1 = alpha * a1[r];
                    *y1 = static_cast<TY>(beta == 0.0 ? v1 : v1 + beta * static_cast<double>(*y1));
                }
            }
    }
}

// Pass 1 of y = M^T x: work[chunk][c][r] = sum over the chunk's 256 rows i of M[i][c] x[i][r].
template <typename TM, typename TX, int NR>
__global__ __launch_bounds__(256) void k_gemv_t_part(int64_t rows, int64_t cols,
                                                     const TM *__restrict__ Mat, int64_t ldm,
                                                     const TX *__restrict__ x, int64_t ldx,
                                                     double *work, int nrhs) {
    __shared__ double xs[256][NR];
    const int64_t i0 = static_cast<int64_t>(blockIdx.y) * 256;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const int cnt = static_cast<int>((rows - i0) < 256 ? (rows - i0) : 256);
    for (int e = threadIdx.x; e < 256 * NR; e += 256) {
        const int i = e / NR, r = e % NR;
        xs[i][r] = (i < cnt && r < nrhs) ? static_cast<double>(x[(i0 + i) * ldx + r]) : 0.0;
    }
    __syncthreads();
    if (c >= cols) return;
    double acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = 0.0;
    const TM *col = Mat + i0 * ldm + c;
    for (int i = 0; i < cnt; ++i) {
        const double m = static_cast<double>(col[i * ldm]);
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r] += m * xs[i][r];
    }
    double *w = work + (static_cast<int64_t>(blockIdx.y) * cols + c) * nrhs;
    for (int r = 0; r < nrhs; ++r) w[r] = acc[r];
}

template <typename TY>
__global__ void k_gemv_t_sum(int64_t chunks, int64_t cols, const double *work, TY *y, int64_t ldy,
                             int nrhs) {
    const int64_t total = cols * nrhs;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t c = e / nrhs, r = e % nrhs;
        double s = 0.0;
        for (int64_t k = 0; k < chunks; ++k) s += work[(k * cols + c) * nrhs + r];
        y[c * ldy + r] = static_cast<TY>(s);
    }
}

__device__ inline void atomic_max_nonneg(double *addr, double v) {
    atomicMax(reinterpret_cast<unsigned long long *>(addr),
              static_cast<unsigned long long>(__double_as_longlong(v)));
}

// norms[r] = max(norms[r], max_i |v[i][r]|); grid.y = r.
__global__ __launch_bounds__(256) void k_colmax(const double *v, int64_t ld, int64_t n,
                                                double *norms) {
    const int r = blockIdx.y;
    double m = 0.0;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        m = fmax(m, fabs(v[i * ld + r]));
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) atomic_max_nonneg(norms + r, m);
}

// out[0] = max(out[0], max_i sum_j |A[i][j]|); one wave per row.
__global__ __launch_bounds__(256) void k_norm_inf(const double *A, int64_t lda, int64_t n,
                                                  double *out) {
    const int lane = threadIdx.x & 63;
    const int64_t row = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    double s = 0.0;
    for (int64_t c = lane; c < n; c += 64) s += fabs(A[row * lda + c]);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) atomic_max_nonneg(out, s);
}

template <typename TS>
__global__ void k_axpby_2d(const TS *d, int64_t ldd, double *x, int64_t ldx, int64_t n, int nrhs,
                           double beta) {
    const int64_t total = n * nrhs;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t i = e / nrhs, r = e % nrhs;
        const double v = static_cast<double>(d[i * ldd + r]);
        double *p = x + i * ldx + r;
        *p = (beta == 0.0) ? v : beta * (*p) + v;
    }
}

__global__ void k_fill_f64(double *p, int64_t count, double value) {
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < count;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[e] = value;
}

int grid_for(int64_t total, int threads) {
    int64_t g = (total + threads - 1) / threads;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return static_cast<int>(g);
}

}  // namespace

template <typename T, int MODE>
hipError_t trsv_full_launch(const T *LU, int64_t ld, int64_t n, const T *B, T *X, int64_t ldx,
                            int nr, int *sync, int epoch, hipStream_t s) {
    const int nblk = static_cast<int>((n + SB - 1) / SB);
    hipLaunchKernelGGL(k_trsv_reset, dim3(1), dim3(1), 0, s, sync);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int *flags = sync + 2, *err = sync + 1;
    if (nr <= 1)
        hipLaunchKernelGGL((k_trsv_persistent<T, MODE, 1>), dim3(nblk), dim3(256), 0, s, LU, ld, n,
                           B, X, ldx, nr, sync, flags, epoch, err);
    else if (nr <= 4)
        hipLaunchKernelGGL((k_trsv_persistent<T, MODE, 4>), dim3(nblk), dim3(256), 0, s, LU, ld, n,
                           B, X, ldx, nr, sync, flags, epoch, err);
    else
        hipLaunchKernelGGL((k_trsv_persistent<T, MODE, 16>), dim3(nblk), dim3(256), 0, s, LU, ld,
                           n, B, X, ldx, nr, sync, flags, epoch, err);
    return hipGetLastError();
}

template <typename T>
hipError_t trsv_full(int mode, const T *LU, int64_t ld, int64_t n, const T *B, T *X, int64_t ldx,
                     int nr, int *sync, int epoch, hipStream_t s) {
    if (nr < 1 || nr > 16 || n < 1) return hipErrorInvalidValue;
    switch (mode) {
    case 0: return trsv_full_launch<T, 0>(LU, ld, n, B, X, ldx, nr, sync, epoch, s);
    case 1: return trsv_full_launch<T, 1>(LU, ld, n, B, X, ldx, nr, sync, epoch, s);
    case 2: return trsv_full_launch<T, 2>(LU, ld, n, B, X, ldx, nr, sync, epoch, s);
    case 3: return trsv_full_launch<T, 3>(LU, ld, n, B, X, ldx, nr, sync, epoch, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t trsv_step(int mode, const T *LU, int64_t ld, int64_t n, int64_t blk, T *Y, T *X,
                     int64_t ldyx, int nr, const int *abort, hipStream_t s) {
    if (nr < 1 || nr > 16 || blk * SB >= n) return hipErrorInvalidValue;
    switch (mode) {
    case 0: return trsv_launch<T, 0>(LU, ld, n, blk, Y, X, ldyx, nr, abort, s);
    case 1: return trsv_launch<T, 1>(LU, ld, n, blk, Y, X, ldyx, nr, abort, s);
    case 2: return trsv_launch<T, 2>(LU, ld, n, blk, Y, X, ldyx, nr, abort, s);
    case 3: return trsv_launch<T, 3>(LU, ld, n, blk, Y, X, ldyx, nr, abort, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename TM, typename TX, typename TY>
hipError_t gemv_n(int64_t rows, int64_t cols, double alpha, const TM *Mat, int64_t ldm,
                  const TX *x, int64_t ldx, double beta, TY *y, int64_t ldy, int nrhs,
                  hipStream_t s) {
    if (rows <= 0 || nrhs <= 0) return hipSuccess;
    if (nrhs > 16) return hipErrorInvalidValue;
    const int64_t grid = (rows + 7) / 8;
    if (nrhs == 1)
        hipLaunchKernelGGL((k_gemv_n<TM, TX, TY, 1>), dim3(static_cast<unsigned>(grid)), dim3(256),
                           0, s, rows, cols, alpha, Mat, ldm, x, ldx, beta, y, ldy, nrhs);
    else if (nrhs <= 4)
        hipLaunchKernelGGL((k_gemv_n<TM, TX, TY, 4>), dim3(static_cast<unsigned>(grid)), dim3(256),
                           0, s, rows, cols, alpha, Mat, ldm, x, ldx, beta, y, ldy, nrhs);
    else
        hipLaunchKernelGGL((k_gemv_n<TM, TX, TY, 16>), dim3(static_cast<unsigned>(grid)),
                           dim3(256), 0, s, rows, cols, alpha, Mat, ldm, x, ldx, beta, y, ldy,
                           nrhs);
    return hipGetLastError();
}

template <typename TM, typename TX, typename TY>
hipError_t gemv_t(int64_t rows, int64_t cols, const TM *Mat, int64_t ldm, const TX *x,
                  int64_t ldx, TY *y, int64_t ldy, int nrhs, double *work, hipStream_t s) {
    if (cols <= 0 || nrhs <= 0) return hipSuccess;
    if (nrhs > 16 || rows <= 0) return hipErrorInvalidValue;
    const int64_t chunks = (rows + 255) / 256;
    dim3 grid(static_cast<unsigned>((cols + 255) / 256), static_cast<unsigned>(chunks));
    if (nrhs == 1)
        hipLaunchKernelGGL((k_gemv_t_part<TM, TX, 1>), grid, dim3(256), 0, s, rows, cols, Mat, ldm,
                           x, ldx, work, nrhs);
    else if (nrhs <= 4)
        hipLaunchKernelGGL((k_gemv_t_part<TM, TX, 4>), grid, dim3(256), 0, s, rows, cols, Mat, ldm,
                           x, ldx, work, nrhs);
    else
        hipLaunchKernelGGL((k_gemv_t_part<TM, TX, 16>), grid, dim3(256), 0, s, rows, cols, Mat,
                           ldm, x, ldx, work, nrhs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gemv_t_sum<TY>, dim3(grid_for(cols * nrhs, 256)), dim3(256), 0, s, chunks,
                       cols, work, y, ldy, nrhs);
    return hipGetLastError();
}

hipError_t colmax_abs(const double *v, int64_t ld, int64_t n, int nrhs, double *norms,
                      hipStream_t s) {
    if (n <= 0 || nrhs <= 0) return hipSuccess;
    int g = grid_for(n, 256);
    if (g > 256) g = 256;
    hipLaunchKernelGGL(k_colmax, dim3(g, nrhs), dim3(256), 0, s, v, ld, n, norms);
    return hipGetLastError();
}

hipError_t norm_inf(const double *A, int64_t lda, int64_t n, double *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_norm_inf, dim3(static_cast<unsigned>((n + 3) / 4)), dim3(256), 0, s, A,
                       lda, n, out);
    return hipGetLastError();
}

template <typename TS>
hipError_t axpby_2d(const TS *d, int64_t ldd, double *x, int64_t ldx, int64_t n, int nrhs,
                    double beta, hipStream_t s) {
    if (n <= 0 || nrhs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_axpby_2d<TS>, dim3(grid_for(n * nrhs, 256)), dim3(256), 0, s, d, ldd, x,
                       ldx, n, nrhs, beta);
    return hipGetLastError();
}

hipError_t fill_f64(double *p, int64_t count, double value, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(count, 256)), dim3(256), 0, s, p, count, value);
    return hipGetLastError();
}

template hipError_t trsv_full<double>(int, const double *, int64_t, int64_t, const double *,
                                      double *, int64_t, int, int *, int, hipStream_t);
template hipError_t trsv_full<float>(int, const float *, int64_t, int64_t, const float *, float *,
                                     int64_t, int, int *, int, hipStream_t);
template hipError_t trsv_step<double>(int, const double *, int64_t, int64_t, int64_t, double *,
                                      double *, int64_t, int, const int *, hipStream_t);
template hipError_t trsv_step<float>(int, const float *, int64_t, int64_t, int64_t, float *,
                                     float *, int64_t, int, const int *, hipStream_t);
template hipError_t gemv_n<double, double, double>(int64_t, int64_t, double, const double *,
                                                   int64_t, const double *, int64_t, double,
                                                   double *, int64_t, int, hipStream_t);
template hipError_t gemv_n<float, float, double>(int64_t, int64_t, double, const float *, int64_t,
                                                 const float *, int64_t, double, double *, int64_t,
                                                 int, hipStream_t);
template hipError_t gemv_t<double, double, double>(int64_t, int64_t, const double *, int64_t,
                                                   const double *, int64_t, double *, int64_t, int,
                                                   double *, hipStream_t);
template hipError_t gemv_t<float, double, float>(int64_t, int64_t, const float *, int64_t,
                                                 const double *, int64_t, float *, int64_t, int,
                                                 double *, hipStream_t);
template hipError_t axpby_2d<double>(const double *, int64_t, double *, int64_t, int64_t, int,
                                     double, hipStream_t);
template hipError_t axpby_2d<float>(const float *, int64_t, double *, int64_t, int64_t, int, double,
                                    hipStream_t);

}  // namespace rmge
