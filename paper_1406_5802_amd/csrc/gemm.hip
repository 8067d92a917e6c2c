// Dense products on the matrix cores of gfx950.
//
// Three places of the method are dense contractions and run here:
//   * the preprocessing product M = A G with a Gaussian multiplier
//     (Fact faprepr; 2n^3 - n^2 flops, the cost the paper states in Section 6);
//   * the two off-diagonal solves of each block step of eq. eqgenp,
//     B^{-1} C and D B^{-1}, done as products with the explicit inverses of
//     the pivot block's triangular factors;
//   * the Schur-complement update S = E - (D B^{-1})(B^{-1} C) of eq. eqgenp.
//
// Kernel: C = alpha A B + beta C, row-major, one workgroup of four waves per
// output tile, each wave a 64 x 64 sub-tile made of 16 x 16 MFMA blocks
// (v_mfma_f64_16x16x4_f64 or v_mfma_f32_16x16x4_f32).  K advances in chunks of
// 16 through double-buffered LDS (A stored m-major, B k-major, one element of
// padding per row), with the next chunk's global loads issued before the
// current chunk's MFMAs.  Workgroup ids are remapped so that each XCD (ids
// are dealt round-robin over the 8 XCDs) gets a contiguous run of tiles, and
// runs are ordered in groups of 8 tile-rows, so the operand panels a wave of
// workgroups touches stay in that XCD's L2.
//
// Bound: MFMA (2 flops per multiply-add).  The product's tile is chosen for
// large K; the Schur update (K = panel width) uses smaller tiles and more
// workgroups per CU so that reading and writing C overlaps the MFMAs.
#include "bf16.h"
#include "mfma.h"
#include "rmge_impl.h"

namespace rmge {
namespace {

__device__ inline void tile_coords(int bid, int tiles_m, int tiles_n, int &tm, int &tn) {
    const int tiles = tiles_m * tiles_n;
    const int q = tiles / 8, r = tiles % 8;
    const int x = bid % 8, i = bid / 8;
    const int logical = x * q + (x < r ? x : r) + i;
    const int G = 8;
    const int per_group = G * tiles_n;
    const int g = logical / per_group;
    const int first = g * G;
    const int gs = (tiles_m - first) < G ? (tiles_m - first) : G;
    const int within = logical - g * per_group;
    tm = first + within % gs;
    tn = within / gs;
}

// One BM x BN output tile (tm, tn) of C = alpha A B + beta C with bounds checks.
// T: arithmetic type, TA / TB: storage types of A and B (a double A may feed a
// float product, a float B a double one).
template <typename T, typename TA, int BM, int BN, int WGM, int WGN, int BK, typename TB = T>
__device__ inline void gemm_tile(int M, int N, int K, T alpha, const TA *A, int64_t lda,
                                 const TB *B, int64_t ldb, T beta, T *C, int64_t ldc,
                                 double *absmax, int tm, int tn) {
    constexpr int NT = WGM * WGN * 64;
    constexpr int WM = BM / WGM, WN = BN / WGN;
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int A_PER = BM * BK / NT;
    constexpr int B_PER = BK * BN / NT;
    constexpr int LDA_S = BK + 1;
    constexpr int LDB_S = BN + 1;
    static_assert(A_PER * NT == BM * BK && B_PER * NT == BK * BN, "tile/threads mismatch");
    using acc_t = typename Mma<T>::acc;

    __shared__ T As[2][BM * LDA_S];
    __shared__ T Bs[2][BK * LDB_S];

    const int m0 = tm * BM, n0 = tn * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;

    acc_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    TA ra[A_PER];
    T rb[B_PER];
    auto load = [&](int k0) {
#pragma unroll
        for (int p = 0; p < A_PER; ++p) {
            const int e = tid + p * NT;
            const int m = m0 + e / BK, k = k0 + e % BK;
            ra[p] = (m < M && k < K) ? A[static_cast<int64_t>(m) * lda + k] : TA(0);
        }
#pragma unroll
        for (int p = 0; p < B_PER; ++p) {
            const int e = tid + p * NT;
            const int k = k0 + e / BN, n = n0 + e % BN;
            rb[p] = (k < K && n < N) ? static_cast<T>(B[static_cast<int64_t>(k) * ldb + n]) : T(0);
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int p = 0; p < A_PER; ++p) {
            const int e = tid + p * NT;
            As[buf][(e / BK) * LDA_S + e % BK] = static_cast<T>(ra[p]);
        }
#pragma unroll
        for (int p = 0; p < B_PER; ++p) {
            const int e = tid + p * NT;
            Bs[buf][(e / BN) * LDB_S + e % BN] = rb[p];
        }
    };

    const int nk = (K + BK - 1) / BK;
    if (nk > 0) {
        load(0);
        store(0);
    }
    __syncthreads();
    const int arow = wm * WM + (lane & 15);
    const int bcol = wn * WN + (lane & 15);
    const int ksub = lane >> 4;
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) load((kt + 1) * BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            T af[TM], bf[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) af[i] = As[cur][(arow + i * 16) * LDA_S + kk + ksub];
#pragma unroll
            for (int j = 0; j < TN; ++j) bf[j] = Bs[cur][(kk + ksub) * LDB_S + bcol + j * 16];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] = Mma<T>::step(af[i], bf[j], acc[i][j]);
        }
        if (kt + 1 < nk) store(cur ^ 1);
        __syncthreads();
    }

    const int crow0 = m0 + wm * WM;
    const int ccol0 = n0 + wn * WN + (lane & 15);
    double vmax = 0.0;
    const bool rd = beta != T(0);
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        // a row of sub-tiles' C values in flight at once (only when beta != 0)
        T cv[TN][4];
        if (rd) {
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = crow0 + i * 16 + Mma<T>::row(lane, r), col = ccol0 + j * 16;
                    cv[j][r] = load_if(C, static_cast<int64_t>(row) * ldc + col, row < M && col < N);
                }
        }
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = crow0 + i * 16 + Mma<T>::row(lane, r), col = ccol0 + j * 16;
                if (row < M && col < N) {
                    const T v = alpha * acc[i][j][r];
                    const T out = rd ? v + beta * cv[j][r] : v;
                    C[static_cast<int64_t>(row) * ldc + col] = out;
                    vmax = fmax(vmax, fabs(static_cast<double>(out)));
                }
            }
    }
    if (absmax != nullptr) {  // max |C| for the growth statistic, one atomic per wave
        for (int off = 32; off > 0; off >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, off));
        if (lane == 0)
            atomicMax(reinterpret_cast<unsigned long long *>(absmax),
                      static_cast<unsigned long long>(__double_as_longlong(vmax)));
    }
}

template <typename T, typename TA, int BM, int BN, int WGM, int WGN, int BK = 16, int MINB = 2>
__global__ __launch_bounds__(WGM *WGN * 64, MINB) void k_gemm(int M, int N, int K, T alpha,
                                                           const TA *A, int64_t lda, const T *B,
                                                           int64_t ldb, T beta, T *C, int64_t ldc,
                                                           const int *abort, double *absmax) {
    if (abort != nullptr && *abort != 0) return;
    const int tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
    int tm, tn;
    tile_coords(blockIdx.x, tiles_m, tiles_n, tm, tn);
    gemm_tile<T, TA, BM, BN, WGM, WGN, BK>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, absmax,
                                           tm, tn);
}

// Batched products M_s = A_s G_s of many square systems of uneven order (A in
// FP64, rounded to FP32 on load; G and M in FP32; each row-major with
// ld = n_s).  Tiles of all systems form one index space: tile_start[s] is the
// first tile of system s (ceil(n_s / 64)^2 tiles, row-major over the tile
// grid), tile_start[count] the total; a workgroup finds its system by binary
// search.  G_s starts at g_off[s] of G, M_s at m_off[s] of M, A_s at a_off[s].
__global__ __launch_bounds__(256, 2) void k_batch_gemm(int count, const int *__restrict__ tile_start,
                                                       const int *__restrict__ nsys,
                                                       const int64_t *__restrict__ a_off,
                                                       const int64_t *__restrict__ g_off,
                                                       const int64_t *__restrict__ m_off,
                                                       const double *A, const float *G, float *M) {
    const int t = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {  // last s with tile_start[s] <= t
        const int mid = (lo + hi + 1) >> 1;
        if (tile_start[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const int s = lo, n = nsys[s];
    const int tiles = (n + 63) / 64, local = t - tile_start[s];
    gemm_tile<float, double, 64, 64, 2, 2, 16>(n, n, n, 1.0f, A + a_off[s], n, G + g_off[s], n,
                                               0.0f, M + m_off[s], n, nullptr, local / tiles,
                                               local % tiles);
}

// The same index space in FP64 for the systems that fall back to FP64 factors:
// M_s = A_s G_s with G_s's FP32 values taken exactly as doubles, only for the
// systems whose flag (flag[sys[s]], sys: the system's index in the caller's
// order) is set; the other tiles' workgroups return at once.
__global__ __launch_bounds__(256, 2) void k_batch_gemm64(int count,
                                                         const int *__restrict__ tile_start,
                                                         const int *__restrict__ nsys,
                                                         const int *__restrict__ sys,
                                                         const int *__restrict__ flag,
                                                         const int64_t *__restrict__ a_off,
                                                         const int64_t *__restrict__ g_off,
                                                         const int64_t *__restrict__ m_off,
                                                         const double *A, const float *G,
                                                         double *M) {
    const int t = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tile_start[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const int s = lo;
    if (flag[sys[s]] == 0) return;
    const int n = nsys[s];
    const int tiles = (n + 63) / 64, local = t - tile_start[s];
    gemm_tile<double, double, 64, 64, 2, 2, 16, float>(n, n, n, 1.0, A + a_off[s], n,
                                                       G + g_off[s], n, 0.0, M + m_off[s], n,
                                                       nullptr, local / tiles, local % tiles);
}

// Interior fast path: M % 128 == N % 128 == K % 16 == 0, lda, ldb, ldc even.
// Same tiling as k_gemm (128 x 128, four 64 x 64 waves, BK = 16), but
//   * no bounds checks in the K loop and no address arithmetic beyond one
//     pointer increment per chunk;
//   * global reads of 8 consecutive elements per thread (16-byte loads);
//   * within a chunk, MFMA step t of lane group s (= lane >> 4) takes
//     k = 4 s + t, a reordering of the chunk's 16-term sum, so each lane's A
//     row segment is 4 consecutive values in LDS (A stored m-major, k
//     contiguous), read as two 16-byte LDS loads; B stays k-major (its
//     16-byte stores stay contiguous) with a row pitch of 132 elements, which
//     puts the four k-rows a wave reads at once on different LDS banks.
// ROLE only names the launch (0: the product M = A H, 1: a Schur update), so
// that the two uses show up as separate kernels in a trace; the code is the same.
template <typename T, typename TA, int MINB, int ROLE>
__global__ __launch_bounds__(256, MINB) void k_gemm_fast(int M, int N, int K, T alpha,
                                                         const TA *__restrict__ A, int64_t lda,
                                                         const T *__restrict__ B, int64_t ldb,
                                                         T beta, T *C, int64_t ldc,
                                                         const int *abort, double *absmax) {
    constexpr int BM = 128, BN = 128, BK = 16, LDK = BK + 2;  // +2: keeps 16-byte alignment
    constexpr int LDN = BN + 4;
    using acc_t = typename Mma<T>::acc;
    __shared__ T As[2][BM * LDK];
    __shared__ T Bs[2][BK * LDN];
    if (abort != nullptr && *abort != 0) return;
    const int tiles_m = M / BM, tiles_n = N / BN;
    int tm, tn;
    tile_coords(blockIdx.x, tiles_m, tiles_n, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;

    // A: thread -> row tid / 2, k = (tid % 2) * 8 .. + 7
    const TA *pa = A + static_cast<int64_t>(m0 + (tid >> 1)) * lda + (tid & 1) * 8;
    // B: thread -> k = tid / 16, n = n0 + (tid % 16) * 8 .. + 7
    const T *pb = B + static_cast<int64_t>(tid >> 4) * ldb + n0 + (tid & 15) * 8;
    const int64_t bstep = static_cast<int64_t>(BK) * ldb;

    TA ra[8];
    T rb[8];
    auto load = [&]() {
#pragma unroll
        for (int u = 0; u < 8; ++u) ra[u] = pa[u];
#pragma unroll
        for (int u = 0; u < 8; ++u) rb[u] = pb[u];
        pa += BK;
        pb += bstep;
    };
    auto store = [&](int buf) {
        T *a = &As[buf][(tid >> 1) * LDK + (tid & 1) * 8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = static_cast<T>(ra[u]);
        T *b = &Bs[buf][(tid >> 4) * LDN + (tid & 15) * 8];
#pragma unroll
        for (int u = 0; u < 8; ++u) b[u] = rb[u];
    };

    acc_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    const int nk = K / BK;
    load();
    store(0);
    __syncthreads();
    const int arow = wm * 64 + (lane & 15);
    const int bcol = wn * 64 + (lane & 15);
    const int k4 = (lane >> 4) * 4;
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) load();
        T af[4][4], bf[4][4];  // [tile][t]
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int t = 0; t < 4; ++t) af[i][t] = As[cur][(arow + 16 * i) * LDK + k4 + t];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int t = 0; t < 4; ++t) bf[j][t] = Bs[cur][(k4 + t) * LDN + bcol + 16 * j];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = Mma<T>::step(af[i][t], bf[j][t], acc[i][j]);
        // FP64: let the scheduler interleave the chunk's LDS reads and writes
        // with its MFMAs (measured: 64 -> 72 TFLOP/s at n = 16384; no gain in FP32)
        if (sizeof(T) == 8) __builtin_amdgcn_iglp_opt(1);
        if (kt + 1 < nk) store(cur ^ 1);
        __syncthreads();
    }

    const int crow0 = m0 + wm * 64;
    const int ccol0 = n0 + wn * 64 + (lane & 15);
    double vmax = 0.0;
    const bool rd = beta != T(0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        // a row of sub-tiles' C values in flight at once (only when beta != 0)
        T cv[4][4];
        if (rd) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    cv[j][r] = C[static_cast<int64_t>(crow0 + i * 16 + Mma<T>::row(lane, r)) * ldc +
                                 ccol0 + j * 16];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = crow0 + i * 16 + Mma<T>::row(lane, r), col = ccol0 + j * 16;
                const T v = alpha * acc[i][j][r];
                const T out = rd ? v + beta * cv[j][r] : v;
                C[static_cast<int64_t>(row) * ldc + col] = out;
                vmax = fmax(vmax, fabs(static_cast<double>(out)));
            }
    }
    if (absmax != nullptr) {
        for (int off = 32; off > 0; off >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, off));
        if (lane == 0)
            atomicMax(reinterpret_cast<unsigned long long *>(absmax),
                      static_cast<unsigned long long>(__double_as_longlong(vmax)));
    }
}

// Interior fast path of the Schur update (K = panel width, beta = 1):
// 64 x 64 tiles of four 32 x 32 waves, four workgroups per CU, with the same
// unchecked addressing, 16-byte loads and k-reordered LDS reads as
// k_gemm_fast.  Needs M % 64 == N % 64 == K % 16 == 0 and even leading
// dimensions.  (Measured at K = 256, n = 16384: FP64 47 -> 62 TFLOP/s,
// FP32 87 -> 103 TFLOP/s.)
template <typename T, int MINB>
__global__ __launch_bounds__(256, MINB) void k_gemm_upd64(int M, int N, int K, T alpha,
                                                          const T *__restrict__ A, int64_t lda,
                                                          const T *__restrict__ B, int64_t ldb,
                                                          T beta, T *C, int64_t ldc,
                                                          const int *abort) {
    constexpr int BM = 64, BN = 64, BK = 16, LDK = BK + 2, LDN = BN + 4;
    using acc_t = typename Mma<T>::acc;
    __shared__ T As[2][BM * LDK];
    __shared__ T Bs[2][BK * LDN];
    if (abort != nullptr && *abort != 0) return;
    int tm, tn;
    tile_coords(blockIdx.x, M / BM, N / BN, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    // A: row tid / 4, k (tid % 4) * 4 .. + 3;  B: k tid / 16, n (tid % 16) * 4 .. + 3
    const T *pa = A + static_cast<int64_t>(m0 + (tid >> 2)) * lda + (tid & 3) * 4;
    const T *pb = B + static_cast<int64_t>(tid >> 4) * ldb + n0 + (tid & 15) * 4;
    const int64_t bstep = static_cast<int64_t>(BK) * ldb;
    T ra[4], rb[4];
    auto load = [&]() {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            ra[u] = pa[u];
            rb[u] = pb[u];
        }
        pa += BK;
        pb += bstep;
    };
    auto store = [&](int buf) {
        T *a = &As[buf][(tid >> 2) * LDK + (tid & 3) * 4];
        T *b = &Bs[buf][(tid >> 4) * LDN + (tid & 15) * 4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] = ra[u];
            b[u] = rb[u];
        }
    };
    acc_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
    const int nk = K / BK;
    load();
    store(0);
    __syncthreads();
    const int arow = wm * 32 + (lane & 15), bcol = wn * 32 + (lane & 15);
    const int k4 = (lane >> 4) * 4;
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) load();
        T af[2][4], bf[2][4];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int t = 0; t < 4; ++t) af[i][t] = As[cur][(arow + 16 * i) * LDK + k4 + t];
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int t = 0; t < 4; ++t) bf[j][t] = Bs[cur][(k4 + t) * LDN + bcol + 16 * j];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = Mma<T>::step(af[i][t], bf[j][t], acc[i][j]);
        if (kt + 1 < nk) store(cur ^ 1);
        __syncthreads();
    }
    const int crow0 = m0 + wm * 32, ccol0 = n0 + wn * 32 + (lane & 15);
    auto cptr = [&](int i, int j, int r) {
        return C + static_cast<int64_t>(crow0 + i * 16 + Mma<T>::row(lane, r)) * ldc + ccol0 +
               j * 16;
    };
    if (beta == T(0)) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) *cptr(i, j, r) = alpha * acc[i][j][r];
    } else {
        // all of the tile's C values in flight at once, then the stores
        T cv[2][2][4];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) cv[i][j][r] = *cptr(i, j, r);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    *cptr(i, j, r) = alpha * acc[i][j][r] + beta * cv[i][j][r];
    }
}

template <typename T, typename TA, int BM, int BN, int WGM, int WGN, int MINB>
hipError_t launch(int m, int n, int k, T alpha, const TA *A, int64_t lda, const T *B, int64_t ldb,
                  T beta, T *C, int64_t ldc, const int *abort, double *absmax, hipStream_t s) {
    const int64_t tiles = static_cast<int64_t>((m + BM - 1) / BM) * ((n + BN - 1) / BN);
    hipLaunchKernelGGL((k_gemm<T, TA, BM, BN, WGM, WGN, 16, MINB>),
                       dim3(static_cast<unsigned>(tiles)), dim3(WGM * WGN * 64), 0, s, m, n, k,
                       alpha, A, lda, B, ldb, beta, C, ldc, abort, absmax);
    return hipGetLastError();
}

// Tile shapes measured on MI355X (n = 16384):
//   product (large K): 128 x 128, four 64 x 64 waves, two workgroups per CU
//     (interior kernel: FP64 71 TFLOP/s, FP32 128 TFLOP/s);
//   Schur update (K = panel width): 64 x 64 tiles of four 32 x 32 waves,
//     four workgroups per CU (interior kernel at K = 256: FP64 62, FP32 103
//     TFLOP/s); ragged shapes fall back to the checked kernel (FP32: 128 x 128
//     tiles of eight 32 x 64 waves).
template <typename T, typename TA>
hipError_t run_gemm(int shape, int64_t M, int64_t N, int64_t K, T alpha, const TA *A, int64_t lda,
                    const T *B, int64_t ldb, T beta, T *C, int64_t ldc, const int *abort,
                    double *absmax, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (M > INT32_MAX || N > INT32_MAX || K > INT32_MAX) return hipErrorInvalidValue;
    const int m = static_cast<int>(M), n = static_cast<int>(N), k = static_cast<int>(K);
    if (shape == kGemmProduct) {
        const bool fits = m % 128 == 0 && n % 128 == 0 && k % 16 == 0 && k > 0 && lda % 2 == 0 &&
                          ldb % 2 == 0;
        if (fits) {
            const int64_t tiles = static_cast<int64_t>(m / 128) * (n / 128);
            hipLaunchKernelGGL((k_gemm_fast<T, TA, 2, 0>), dim3(static_cast<unsigned>(tiles)),
                               dim3(256), 0, s, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                               abort, absmax);
            return hipGetLastError();
        }
        return launch<T, TA, 128, 128, 2, 2, 2>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                                                abort, absmax, s);
    }
    // Schur update.  FP32 trailing blocks of 4096 and more: the 128 x 128
    // kernel (measured at K = 256: 110 against 84-100 TFLOP/s for 64 x 64
    // tiles); smaller blocks, and FP64 (where 64 x 64 tiles win below the
    // largest blocks), use k_gemm_upd64.
    const bool fits128 = m % 128 == 0 && n % 128 == 0 && k % 16 == 0 && k > 0 && lda % 2 == 0 &&
                         ldb % 2 == 0;
    if (sizeof(T) == 4 && sizeof(TA) == 4 && fits128 && m >= 4096 && n >= 4096) {
        const int64_t tiles = static_cast<int64_t>(m / 128) * (n / 128);
        hipLaunchKernelGGL((k_gemm_fast<T, TA, 2, 1>), dim3(static_cast<unsigned>(tiles)),
                           dim3(256), 0, s, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, abort,
                           absmax);
        return hipGetLastError();
    }
    const bool fits64 = m % 64 == 0 && n % 64 == 0 && k % 16 == 0 && k > 0 && lda % 2 == 0 &&
                        ldb % 2 == 0 && absmax == nullptr && sizeof(TA) == sizeof(T);
    if (fits64) {
        const int64_t tiles = static_cast<int64_t>(m / 64) * (n / 64);
        hipLaunchKernelGGL((k_gemm_upd64<T, 4>), dim3(static_cast<unsigned>(tiles)), dim3(256), 0,
                           s, m, n, k, alpha, reinterpret_cast<const T *>(A), lda, B, ldb, beta, C,
                           ldc, abort);
        return hipGetLastError();
    }
    if (sizeof(T) == 8)
        return launch<T, TA, 64, 64, 2, 2, 4>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, abort,
                                              absmax, s);
    return launch<T, TA, 128, 128, 4, 2, 1>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, abort,
                                            absmax, s);
}

}  // namespace

hipError_t gemm_f64(int shape, int64_t M, int64_t N, int64_t K, double alpha, const double *A,
                    int64_t lda, const double *B, int64_t ldb, double beta, double *C, int64_t ldc,
                    const int *abort, hipStream_t s, double *absmax) {
    return run_gemm<double, double>(shape, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, abort,
                                    absmax, s);
}

hipError_t gemm_f32(int shape, int64_t M, int64_t N, int64_t K, float alpha, const float *A,
                    int64_t lda, const float *B, int64_t ldb, float beta, float *C, int64_t ldc,
                    const int *abort, hipStream_t s, double *absmax) {
    return run_gemm<float, float>(shape, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, abort,
                                  absmax, s);
}

hipError_t gemm_f32_a64(int shape, int64_t M, int64_t N, int64_t K, float alpha, const double *A,
                        int64_t lda, const float *B, int64_t ldb, float beta, float *C,
                        int64_t ldc, const int *abort, hipStream_t s, double *absmax) {
    return run_gemm<float, double>(shape, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, abort,
                                   absmax, s);
}


// ---------------------------------------------------------------------------
// The product M = A H of the FP32 path on the BF16 matrix cores (precision
// RMGE_F32_BF16X2).  H is a random multiplier chosen by the library, so it is
// drawn and then rounded to BF16, which makes it exact in BF16 (the same
// rounded H is used by the solves); A is split into two BF16 terms,
// A = A_h + A_l + O(2^-18 |A|).  Then M = A_h H + A_l H: one GEMM over both
// terms with FP32 accumulation, on v_mfma_f32_16x16x32_bf16 (eight times the
// FP32 rate per instruction), leaving a product error of the FP32 product's
// order, far below the FP32 factorization's own.
//
// Operands are K-contiguous: A_h, A_l row-major (rows x ldk) and H stored
// transposed (Ht[j][k] = H[k][j]), all zero-padded to whole 256-row tiles and
// 32-wide K chunks, so no load is checked; only the C store is.  One
// workgroup per CU: a 256 x 256 tile, sixteen waves of 64 x 64 (4 x 4 MFMA
// tiles of 16 x 16; 256 x 256 measured 48 % of the BF16 peak against 36 % for
// 128 x 128, which moves 1.6 times the operand bytes per flop);
// lane (lo, hi) = (l & 15, l >> 4) supplies A[m0 + lo][8 hi .. +7]
// and Ht[n0 + lo][8 hi .. +7] of a 32-wide chunk (any k assignment shared by
// both operands gives the same product) and receives C[4 hi + r][lo].  Chunks
// are double-buffered in LDS with the next chunk's global loads in flight.
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(1024, 1) void k_gemm_bf16x2(int M, int N, int Kp,
                                                         const uint16_t *__restrict__ Ah,
                                                         const uint16_t *__restrict__ Al,
                                                         int64_t lda,
                                                         const uint16_t *__restrict__ Ht,
                                                         int64_t ldh, float *C, int64_t ldc,
                                                         double *absmax) {
    constexpr int BM = 256, BN = 256, BK = 32, PAD = 8, LDK = BK + PAD;  // LDS row: 80 bytes
    __shared__ __attribute__((aligned(16))) uint16_t sa[2][2][BM][LDK];
    __shared__ __attribute__((aligned(16))) uint16_t sb[2][BN][LDK];
    const int tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
    int tm, tn;
    tile_coords(blockIdx.x, tiles_m, tiles_n, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lo = lane & 15, hi = lane >> 4;
    const int wm = wave >> 2, wn = wave & 3;
    // global -> LDS: 256 rows x 4 pieces of 8 values per operand, one piece a thread
    const int pr = tid >> 2, pk = 8 * (tid & 3);
    const uint16_t *gah = Ah + static_cast<int64_t>(m0 + pr) * lda + pk;
    const uint16_t *gal = Al + static_cast<int64_t>(m0 + pr) * lda + pk;
    const uint16_t *gb = Ht + static_cast<int64_t>(n0 + pr) * ldh + pk;
    uint4 r0, r1, r2;  // the next chunk's global loads, in flight during this chunk
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    r0 = *reinterpret_cast<const uint4 *>(gah);
    r1 = *reinterpret_cast<const uint4 *>(gal);
    r2 = *reinterpret_cast<const uint4 *>(gb);
    *reinterpret_cast<uint4 *>(&sa[0][0][pr][pk]) = r0;
    *reinterpret_cast<uint4 *>(&sa[0][1][pr][pk]) = r1;
    *reinterpret_cast<uint4 *>(&sb[0][pr][pk]) = r2;
    __syncthreads();
    int buf = 0;
    for (int k0 = 0; k0 < Kp; k0 += BK) {
        const bool more = k0 + BK < Kp;
        if (more) {
            r0 = *reinterpret_cast<const uint4 *>(gah + k0 + BK);
            r1 = *reinterpret_cast<const uint4 *>(gal + k0 + BK);
            r2 = *reinterpret_cast<const uint4 *>(gb + k0 + BK);
        }
        bf16x8 fb[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            fb[j] = *reinterpret_cast<const bf16x8 *>(&sb[buf][wn * 64 + j * 16 + lo][8 * hi]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const bf16x8 fh =
                *reinterpret_cast<const bf16x8 *>(&sa[buf][0][wm * 64 + i * 16 + lo][8 * hi]);
            const bf16x8 fl =
                *reinterpret_cast<const bf16x8 *>(&sa[buf][1][wm * 64 + i * 16 + lo][8 * hi]);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fh, fb[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fl, fb[j], acc[i][j], 0, 0, 0);
            }
        }
        if (more) {
            *reinterpret_cast<uint4 *>(&sa[buf ^ 1][0][pr][pk]) = r0;
            *reinterpret_cast<uint4 *>(&sa[buf ^ 1][1][pr][pk]) = r1;
            *reinterpret_cast<uint4 *>(&sb[buf ^ 1][pr][pk]) = r2;
        }
        __syncthreads();
        buf ^= 1;
    }
    double vmax = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = m0 + wm * 64 + i * 16 + 4 * hi + q;
                const int col = n0 + wn * 64 + j * 16 + lo;
                if (row < M && col < N) {
                    const float v = acc[i][j][q];
                    C[static_cast<int64_t>(row) * ldc + col] = v;
                    vmax = fmax(vmax, fabs(static_cast<double>(v)));
                }
            }
    if (absmax != nullptr) {
        for (int off = 32; off > 0; off >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, off));
        if (lane == 0)
            atomicMax(reinterpret_cast<unsigned long long *>(absmax),
                      static_cast<unsigned long long>(__double_as_longlong(vmax)));
    }
}

}  // namespace

namespace {


// A (n x n, lda, FP64) -> A_h = bf16(A), A_l = bf16(A - A_h) (n x ldk each,
// ldk >= round_up(n, 8); a column n written as zero when n is odd, the rest
// of the padding left as allocated, zero).  Two consecutive columns a thread,
// so a wave reads 1 KB and writes 256 bytes per term contiguously (16-byte
// loads when A's rows are 16-byte aligned, `vec`); rows by blockIdx.y with a
// stride for n beyond the grid's y limit.
__global__ __launch_bounds__(256) void k_split_bf16(const double *__restrict__ A, int64_t lda,
                                                    int64_t n, uint16_t *ah, uint16_t *al,
                                                    int64_t ldk, int vec) {
    const int64_t j = 2 * (static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x);
    if (j >= n) return;
    const bool two = j + 1 < n;
    for (int64_t i = blockIdx.y; i < n; i += gridDim.y) {
        const double *p = A + i * lda + j;
        double a[2];
        if (vec && two) {
            const double2 v = *reinterpret_cast<const double2 *>(p);
            a[0] = v.x;
            a[1] = v.y;
        } else {
            a[0] = p[0];
            a[1] = two ? p[1] : 0.0;
        }
        uint32_t h[2], l[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const uint16_t hb = bf16_bits(static_cast<float>(a[u]));
            h[u] = hb;
            l[u] = bf16_bits(static_cast<float>(a[u] - static_cast<double>(bf16_value(hb))));
        }
        *reinterpret_cast<uint32_t *>(ah + i * ldk + j) = h[0] | (h[1] << 16);
        *reinterpret_cast<uint32_t *>(al + i * ldk + j) = l[0] | (l[1] << 16);
    }
}

// H (n x n row-major FP32) rounded to BF16 in place, and its transpose as BF16
// bits into Ht (n x ldk): 32 x 32 tiles through LDS so both sides coalesce.
__global__ __launch_bounds__(256) void k_round_h_bf16(float *H, int64_t n, uint16_t *Ht,
                                                      int64_t ldk) {
    __shared__ uint16_t t[32][33];
    const int64_t r0 = static_cast<int64_t>(blockIdx.y) * 32, c0 = static_cast<int64_t>(blockIdx.x) * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int k = ty; k < 32; k += 8) {
        const int64_t r = r0 + k, c = c0 + tx;
        if (r < n && c < n) {
            const uint16_t h = bf16_bits(H[r * n + c]);
            H[r * n + c] = bf16_value(h);
            t[k][tx] = h;
        }
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int64_t c = c0 + k, r = r0 + tx;  // Ht[c][r] = H[r][c]
        if (r < n && c < n) Ht[c * ldk + r] = t[tx][k];
    }
}

}  // namespace

hipError_t split_bf16(const double *A, int64_t lda, int64_t n, uint16_t *ah, uint16_t *al,
                      int64_t ldk, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (ldk % 8 != 0 || ldk < (n + 7) / 8 * 8) return hipErrorInvalidValue;
    const int64_t gx = (n + 511) / 512, gy = n < 65535 ? n : 65535;
    const int vec = (reinterpret_cast<uintptr_t>(A) % 16 == 0 && lda % 2 == 0) ? 1 : 0;
    hipLaunchKernelGGL(k_split_bf16, dim3(static_cast<unsigned>(gx), static_cast<unsigned>(gy)),
                       dim3(256), 0, s, A, lda, n, ah, al, ldk, vec);
    return hipGetLastError();
}

hipError_t round_h_bf16(float *H, int64_t n, uint16_t *Ht, int64_t ldk, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + 31) / 32;
    if (nb > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_round_h_bf16, dim3(static_cast<unsigned>(nb), static_cast<unsigned>(nb)),
                       dim3(256), 0, s, H, n, Ht, ldk);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Schur update of the split-BF16 path, C <- C - D E (eq. eqgenp with the
// pivot block's solves already applied: D = D U_B^{-1}, E = L_B^{-1} C), on
// the BF16 matrix cores at the FP32 product's accuracy.  Each FP32 value is
// cut into three BF16 terms, x = x_1 + x_2 + x_3 exactly (x_1 = bf16(x),
// x_2 = bf16(x - x_1), x_3 = x - x_1 - x_2: each takes the next 8 bits of
// the 24-bit significand; |x_2| <= 2^-8 |x|, |x_3| <= 2^-17 |x|).  Of the
// nine cross products x_i y_j the six with i + j <= 4 are formed; the three
// left out total at most (2^-24 + 2^-34) |x y|, one unit of FP32 rounding,
// the error FP32 itself makes in rounding each product, while every product
// kept is exact and accumulates in FP32.  Six BF16 instructions do the work
// of one FP32 product at 16 times the FP32 rate.
//
// The accumulators start from C (so the result is C + sum (-D) E with -D
// split), and the terms enter from the largest down.  Operands come from a
// workspace the split kernel fills each step: the terms of -D as rows
// (row i, k contiguous) and those of E transposed (row j = column j of E),
// each term a (rows x ldk) slab, pstride apart; rows beyond M or N may hold
// anything finite (they reach only the outputs that are not stored), k in
// [K, Kp) holds zeros.  One workgroup per CU: a 256 x 256 tile, four waves
// of 128 x 128 (8 x 8 MFMA tiles), one a SIMD, so that each has 512
// registers: a 256-register accumulator, the next chunk's 24 loads and one
// term's fragments of both operands.  The six terms of a 32-wide chunk take
// 120 KB of LDS, so it is single-buffered: the next chunk's global loads are
// in flight during this chunk's 384 MFMAs a wave and are written after a
// barrier.
//
// With NT = 1 the same kernel is the BF16 Schur update of the BF16 factors
// (RMGE_BF16): each operand is rounded once to BF16 (relative error up to
// 2^-9) and the single product x_1 y_1 accumulates in FP32.
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// 16 bytes at byte offset voff + soff of a buffer (soff wave-uniform).
__device__ inline uint4 buf_load16(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    return uint4{v.x, v.y, v.z, v.w};
}

// ws: the NT terms of -D (rows, NT slabs) then those of E^T (NT slabs);
// bytes: its size, below 2^31, so every offset fits a buffer load's 32 bits.
template <int NT>
__global__ __launch_bounds__(256, 1) void k_update_bf16x3(int M, int N, int Kp,
                                                          const uint16_t *__restrict__ ws,
                                                          int bytes, int ldk, int pstride,
                                                          float *C, int64_t ldc,
                                                          const int *abort) {
    constexpr int BM = 256, BN = 256, BK = 32, LDK = BK + 8;  // LDS row: 80 bytes
    __shared__ __attribute__((aligned(16))) uint16_t sa[NT][BM][LDK];
    __shared__ __attribute__((aligned(16))) uint16_t sb[NT][BN][LDK];
    if (abort != nullptr && *abort != 0) return;
    const int tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
    int tm, tn;
    tile_coords(blockIdx.x, tiles_m, tiles_n, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lo = lane & 15, hi = lane >> 4;
    const int wm = wave >> 1, wn = wave & 1;  // 2 x 2 waves of 128 x 128
    // global -> LDS: per term and operand 256 rows x 4 pieces of 8 values;
    // this thread moves rows pr + 64 h, h < 4
    // (buffer loads: one address register an operand, the rest in scalars)
    const int pr = tid >> 2, pk = 8 * (tid & 3);
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t *>(ws), 0, bytes, 0x00020000);
    const int va = 2 * ((m0 + pr) * ldk + pk);
    const int vb = 2 * ((n0 + pr) * ldk + pk + NT * pstride);
    auto soff = [&](int p, int h, int k) { return 2 * (p * pstride + h * 64 * ldk + k); };
    uint4 ra[NT][4], rb[NT][4];
#pragma unroll
    for (int p = 0; p < NT; ++p)
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            ra[p][h] = buf_load16(rs, va, soff(p, h, 0));
            rb[p][h] = buf_load16(rs, vb, soff(p, h, 0));
        }
    // the accumulators start from C; outside M x N they read a clamped
    // (in-range) address and are never stored
    f32x4 acc[8][8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = m0 + wm * 128 + i * 16 + 4 * hi + q;
            const float *crow = C + static_cast<int64_t>(row < M ? row : M - 1) * ldc;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int col = n0 + wn * 128 + j * 16 + lo;
                acc[i][j][q] = crow[col < N ? col : N - 1];
            }
        }
#pragma unroll
    for (int p = 0; p < NT; ++p)
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            *reinterpret_cast<uint4 *>(&sa[p][pr + 64 * h][pk]) = ra[p][h];
            *reinterpret_cast<uint4 *>(&sb[p][pr + 64 * h][pk]) = rb[p][h];
        }
    // drain the C loads here: left pending into the loop, they would make the
    // compiler wait for every load (the next chunk's too) before each chunk's MFMAs
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int k0 = 0; k0 < Kp; k0 += BK) {
        const bool more = k0 + BK < Kp;
        if (more) {
#pragma unroll
            for (int p = 0; p < NT; ++p)
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    ra[p][h] = buf_load16(rs, va, soff(p, h, k0 + BK));
                    rb[p][h] = buf_load16(rs, vb, soff(p, h, k0 + BK));
                }
        }
#pragma unroll
        for (int p = 0; p < NT; ++p) {
            bf16x8 fa[8];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                fa[i] = *reinterpret_cast<const bf16x8 *>(&sa[p][wm * 128 + i * 16 + lo][8 * hi]);
#pragma unroll
            for (int q = 0; p + q < NT; ++q) {
                bf16x8 fb[8];
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    fb[j] =
                        *reinterpret_cast<const bf16x8 *>(&sb[q][wn * 128 + j * 16 + lo][8 * hi]);
#pragma unroll
                for (int i = 0; i < 8; ++i)
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        acc[i][j] =
                            __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
            }
        }
        __syncthreads();
        if (more) {
#pragma unroll
            for (int p = 0; p < NT; ++p)
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    *reinterpret_cast<uint4 *>(&sa[p][pr + 64 * h][pk]) = ra[p][h];
                    *reinterpret_cast<uint4 *>(&sb[p][pr + 64 * h][pk]) = rb[p][h];
                }
        }
        __syncthreads();
    }
    if (m0 + BM <= M && n0 + BN <= N) {
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float *crow = C + static_cast<int64_t>(m0 + wm * 128 + i * 16 + 4 * hi + q) * ldc;
#pragma unroll
                for (int j = 0; j < 8; ++j) crow[n0 + wn * 128 + j * 16 + lo] = acc[i][j][q];
            }
        return;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = m0 + wm * 128 + i * 16 + 4 * hi + q;
                const int col = n0 + wn * 128 + j * 16 + lo;
                if (row < M && col < N) C[static_cast<int64_t>(row) * ldc + col] = acc[i][j][q];
            }
}

// x = t[0] + t[1] + t[2], each a BF16 bit pattern (exact for finite x away
// from the bottom of the exponent range).
__device__ inline void split3(float x, uint16_t &t0, uint16_t &t1, uint16_t &t2) {
    t0 = bf16_bits(x);
    const float r1 = x - bf16_value(t0);
    t1 = bf16_bits(r1);
    t2 = bf16_bits(r1 - bf16_value(t1));
}

// The update's operands: blocks [0, nbd) cut -D (M x K, ldd) into its three
// terms as rows of dp (eight k a thread); the rest cut E (K x N, lde) into
// those of E^T in ep, 32 k x 64 columns a block through LDS so that both the
// row reads and the k-contiguous writes coalesce.  k in [K, Kp) gets zeros.
template <int NT>
__global__ __launch_bounds__(256) void k_split3_panels(const float *__restrict__ D, int64_t ldd,
                                                       int M, const float *__restrict__ E,
                                                       int64_t lde, int N, int K, int Kp,
                                                       uint16_t *dp, uint16_t *ep, int64_t ldk,
                                                       int64_t pstride, int nbd,
                                                       const int *abort) {
    __shared__ float t[32][65];
    if (abort != nullptr && *abort != 0) return;
    const int kc = Kp / 8;  // pieces of eight a row
    if (static_cast<int>(blockIdx.x) < nbd) {
        const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
        const int i = static_cast<int>(e / kc), k = 8 * static_cast<int>(e % kc);
        if (i >= M) return;
        uint16_t v0[8], v1[8], v2[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const float x = k + u < K ? -D[static_cast<int64_t>(i) * ldd + k + u] : 0.f;
            split3(x, v0[u], v1[u], v2[u]);
        }
        uint16_t *o = dp + static_cast<int64_t>(i) * ldk + k;
        *reinterpret_cast<uint4 *>(o) = pack8(v0);
        if (NT == 3) {
            *reinterpret_cast<uint4 *>(o + pstride) = pack8(v1);
            *reinterpret_cast<uint4 *>(o + 2 * pstride) = pack8(v2);
        }
        return;
    }
    const int b = static_cast<int>(blockIdx.x) - nbd;
    const int nbj = (N + 63) / 64;
    const int j0 = (b % nbj) * 64, k0 = (b / nbj) * 32;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
    for (int kk = ty; kk < 32; kk += 4) {
        const int k = k0 + kk, j = j0 + tx;
        t[kk][tx] = (k < K && j < N) ? E[static_cast<int64_t>(k) * lde + j] : 0.f;
    }
    __syncthreads();
    const int jj = threadIdx.x >> 2, c = 8 * (threadIdx.x & 3);
    const int j = j0 + jj;
    if (j >= N) return;
    uint16_t v0[8], v1[8], v2[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) split3(t[c + u][jj], v0[u], v1[u], v2[u]);
    uint16_t *o = ep + static_cast<int64_t>(j) * ldk + k0 + c;
    *reinterpret_cast<uint4 *>(o) = pack8(v0);
    if (NT == 3) {
        *reinterpret_cast<uint4 *>(o + pstride) = pack8(v1);
        *reinterpret_cast<uint4 *>(o + 2 * pstride) = pack8(v2);
    }
}

}  // namespace

hipError_t update_bf16(int terms, int64_t M, int64_t N, int64_t K, const float *D, int64_t ldd,
                       const float *E, int64_t lde, float *C, int64_t ldc, uint16_t *ws,
                       int64_t ldk, int64_t rows, const int *abort, hipStream_t s) {
    if (terms != 1 && terms != 3) return hipErrorInvalidValue;
    if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
    const int64_t Kp = (K + 31) / 32 * 32;
    if (M > INT32_MAX || N > INT32_MAX || ldk % 8 != 0 || ldk < Kp || rows % 256 != 0 ||
        rows < (M + 255) / 256 * 256 || rows < (N + 255) / 256 * 256)
        return hipErrorInvalidValue;
    const int64_t pstride = rows * ldk;
    if (4 * terms * pstride > INT32_MAX) return hipErrorInvalidValue;  // 32-bit buffer offsets
    uint16_t *dp = ws, *ep = ws + terms * pstride;
    const int64_t nbd = (M * (Kp / 8) + 255) / 256;
    const int64_t nbe = ((N + 63) / 64) * (Kp / 32);
    if (nbd + nbe > INT32_MAX) return hipErrorInvalidValue;
    auto split = terms == 3 ? k_split3_panels<3> : k_split3_panels<1>;
    hipLaunchKernelGGL(split, dim3(static_cast<unsigned>(nbd + nbe)), dim3(256), 0, s, D, ldd,
                       static_cast<int>(M), E, lde, static_cast<int>(N), static_cast<int>(K),
                       static_cast<int>(Kp), dp, ep, ldk, pstride, static_cast<int>(nbd), abort);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t tiles = ((M + 255) / 256) * ((N + 255) / 256);
    auto upd = terms == 3 ? k_update_bf16x3<3> : k_update_bf16x3<1>;
    hipLaunchKernelGGL(upd, dim3(static_cast<unsigned>(tiles)), dim3(256), 0, s,
                       static_cast<int>(M), static_cast<int>(N), static_cast<int>(Kp),
                       static_cast<const uint16_t *>(ws), static_cast<int>(4 * terms * pstride),
                       static_cast<int>(ldk), static_cast<int>(pstride), C, ldc, abort);
    return hipGetLastError();
}

hipError_t batch_gemm_f32(int count, int total_tiles, const int *tile_start, const int *nsys,
                          const int64_t *a_off, const int64_t *g_off, const int64_t *m_off,
                          const double *A, const float *G, float *M, hipStream_t s) {
    if (count <= 0 || total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_gemm, dim3(static_cast<unsigned>(total_tiles)), dim3(256), 0, s,
                       count, tile_start, nsys, a_off, g_off, m_off, A, G, M);
    return hipGetLastError();
}

// Y = beta Y + alpha M X for a few right-hand sides (X: cols x nrhs FP64, nrhs <=
// 16) as a skinny product on the FP64 matrix cores: 64 x 16 tiles of four 16 x
// 16 waves, so the 16 columns of X staged in LDS serve 64 rows of M at a time
// (a matrix-vector kernel re-reads all of X for every pair of rows).
template <typename TM>
hipError_t gemm_skinny(int64_t rows, int64_t cols, double alpha, const TM *Mat, int64_t ldm,
                       const double *X, int64_t ldx, double beta, double *Y, int64_t ldy,
                       int nrhs, hipStream_t s) {
    if (rows <= 0 || nrhs <= 0) return hipSuccess;
    if (rows > INT32_MAX || cols > INT32_MAX || nrhs > 16) return hipErrorInvalidValue;
    const int64_t tiles = (rows + 63) / 64;
    hipLaunchKernelGGL((k_gemm<double, TM, 64, 16, 4, 1, 16, 4>),
                       dim3(static_cast<unsigned>(tiles)), dim3(256), 0, s,
                       static_cast<int>(rows), nrhs, static_cast<int>(cols), alpha, Mat, ldm, X,
                       ldx, beta, Y, ldy, nullptr, nullptr);
    return hipGetLastError();
}

template hipError_t gemm_skinny<double>(int64_t, int64_t, double, const double *, int64_t,
                                        const double *, int64_t, double, double *, int64_t, int,
                                        hipStream_t);
template hipError_t gemm_skinny<float>(int64_t, int64_t, double, const float *, int64_t,
                                       const double *, int64_t, double, double *, int64_t, int,
                                       hipStream_t);

hipError_t batch_gemm_f64(int count, int total_tiles, const int *tile_start, const int *nsys,
                          const int *sys, const int *flag, const int64_t *a_off,
                          const int64_t *g_off, const int64_t *m_off, const double *A,
                          const float *G, double *M, hipStream_t s) {
    if (count <= 0 || total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_gemm64, dim3(static_cast<unsigned>(total_tiles)), dim3(256), 0, s,
                       count, tile_start, nsys, sys, flag, a_off, g_off, m_off, A, G, M);
    return hipGetLastError();
}

hipError_t gemm_bf16x2(int64_t M, int64_t N, int64_t Kp, const uint16_t *Ah, const uint16_t *Al,
                       int64_t lda, const uint16_t *Ht, int64_t ldh, float *C, int64_t ldc,
                       hipStream_t s, double *absmax) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (M > INT32_MAX || N > INT32_MAX || Kp > INT32_MAX || Kp % 32 != 0 || lda % 8 != 0 ||
        ldh % 8 != 0 || lda < Kp || ldh < Kp)
        return hipErrorInvalidValue;
    const int64_t tiles = ((M + 255) / 256) * ((N + 255) / 256);
    hipLaunchKernelGGL(k_gemm_bf16x2, dim3(static_cast<unsigned>(tiles)), dim3(1024), 0, s,
                       static_cast<int>(M), static_cast<int>(N), static_cast<int>(Kp), Ah, Al, lda,
                       Ht, ldh, C, ldc, absmax);
    return hipGetLastError();
}

}  // namespace rmge
