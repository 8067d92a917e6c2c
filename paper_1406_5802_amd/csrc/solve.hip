// Triangular solves, back-transformation and refinement residuals.
//
// After M = A H = L U, the solution of A x = b is x = H U^{-1} L^{-1} b
// (Fact faprepr), and its transpose gives the adjoint A^{-T} w =
// L^{-T} U^{-T} H^T w.  Refinement (Section 8.1) needs r = b - A x in FP64.
// Every kernel here streams a matrix once and is bound by HBM bandwidth.
//
// Triangular solves are blocked by 64 rows and run as one persistent launch
// (k_trsv); coupling tiles are read as row segments (coalesced) for plain and
// transposed factors alike.  Their critical path is the chain of 64-row
// blocks, not HBM bandwidth.
#include "mfma.h"
#include "rmge_impl.h"

namespace rmge {
namespace {

constexpr int SB = 64;  // rows per block of the persistent solve
constexpr int SW = 32;  // its two diagonal sub-blocks, applied through their inverses

// Whole triangular solve in one launch.  Workgroups take 64-row blocks in the
// order they start (a ticket from an atomic counter), so every block a
// workgroup waits on belongs to a workgroup that is already running.  Block I
// accumulates the coupling T_IJ y_J of every block J before it, then solves
// its diagonal block through the inverses of its two 32 x 32 sub-blocks
// (x_a = D_a^{-1} s_a; s_b -= C x_a; x_b = D_b^{-1} s_b), three small parallel
// products instead of 64 dependent steps.
//
// Hand-off without flags: the output is pre-filled with a signalling-NaN
// mark that arithmetic never produces; a finished block publishes its values
// with agent-scope atomic stores, and a waiting block polls the values it
// needs with agent-scope atomic loads until none is the mark.  The data is the
// flag, so no fence sits on the chain from one block to the next.  Coupling
// tiles are prefetched one block ahead into registers.  A wait gives up after
// kSpinLimit polls and records an error instead of hanging; the caller
// checks it.
constexpr int kSpinLimit = 1 << 22;

constexpr unsigned long long kMark = 0x7FF4D1A6C0DE0001ull;  // FP64 signalling NaN

__device__ inline double poll_value(const double *p, bool *ready) {
    const unsigned long long b =
        __hip_atomic_load(reinterpret_cast<unsigned long long *>(const_cast<double *>(p)),
                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *ready = (b != kMark);
    return __builtin_bit_cast(double, b);
}

__device__ inline void publish_value(double *p, double v) {
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(p),
                       __builtin_bit_cast(unsigned long long, v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// The last value a thread publishes for a row of several right-hand sides:
// a release store, so a block that sees it (and then fences with acquire)
// also sees the row's other values; waiting blocks poll only this one.
__device__ inline void publish_last(double *p, double v) {
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(p),
                       __builtin_bit_cast(unsigned long long, v), __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// modes: 0 L y = b (unit lower, forward)    1 U y = b (upper, backward)
//        2 U^T y = b (forward)              3 L^T y = b (unit upper, backward)
// Dinv: the compact inverses of the 32 x 32 diagonal sub-blocks of the factor
// the mode uses (L for 0 and 3, U for 1 and 2): row 32 q + i holds row i of
// sub-block q's inverse.  Factors in T; vectors and arithmetic in FP64 (the
// factors are what streams from HBM, so FP32 factors keep their bandwidth
// advantage while the solve itself adds no FP32 rounding).
template <typename T, int MODE, int NR>
__global__ __launch_bounds__(256) void k_trsv(const T *LU, int64_t ld, int64_t n, const T *Dinv,
                                              const double *B, double *X, int64_t ldx, int nr,
                                              int *sync) {
    constexpr bool forward = (MODE == 0 || MODE == 2);
    constexpr bool transposed = (MODE == 2 || MODE == 3);
    // with eight or more right-hand sides the coupling T_IJ y_J runs on the
    // FP64 matrix cores: wave w takes rows 16 w .. 16 w + 15 of the block and a
    // 16-column slab of right-hand sides, the tile staged in LDS in natural
    // order (the lanes' operand layout differs from the load layout)
    constexpr bool kMma = NR >= 8;
    __shared__ T Ts[(transposed || kMma) ? SB : 1][SB + 1];  // staged tile (Ts[row][col])
    __shared__ T Dd[2][SW][SW + 1];                 // sub-block inverses, as applied
    __shared__ T Cp[SW][SW + 1];                    // first-solved sub-block -> second
    __shared__ double ys[SB][NR];
    __shared__ double xs[SB][NR];
    __shared__ int s_ticket, s_fail;
    int *counter = sync, *err = sync + 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) {
        s_ticket = atomicAdd(counter, 1);
        s_fail = 0;
    }
    __syncthreads();
    const int nblk = static_cast<int>((n + SB - 1) / SB);
    const int I = forward ? s_ticket : nblk - 1 - s_ticket;
    const int64_t I0 = static_cast<int64_t>(I) * SB;
    const int bI = static_cast<int>((n - I0) < SB ? (n - I0) : SB);

    // Everything that does not depend on other blocks is loaded before waiting.
    for (int e = tid; e < 2 * SW * SW; e += 256) {
        const int sb = e / (SW * SW), i = (e / SW) % SW, j = e % SW;
        const bool in = (SW * sb + i < bI) && (SW * sb + j < bI);
        const int64_t row = I0 + SW * sb + (transposed ? j : i);
        Dd[sb][i][j] = in ? Dinv[row * SW + (transposed ? i : j)] : T(0);
    }
    for (int e = tid; e < SW * SW; e += 256) {
        const int i = e / SW, j = e % SW;
        int rr, cc;  // block-local position in the packed factors
        if (MODE == 0) { rr = SW + i; cc = j; }       // L_ba
        else if (MODE == 1) { rr = i; cc = SW + j; }  // U_ab
        else if (MODE == 2) { rr = j; cc = SW + i; }  // (U^T)_ba = U_ab^T
        else { rr = SW + j; cc = i; }                 // (L^T)_ab = L_ba^T
        Cp[i][j] = (rr < bI && cc < bI) ? LU[(I0 + rr) * ld + I0 + cc] : T(0);
    }
    const int r = tid >> 2, q = tid & 3;  // tile row r, columns 16 q .. 16 q + 15
    double bval[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c)
        bval[c] = (q == 0 && r < bI && c < nr) ? B[(I0 + r) * ldx + c] : 0.0;
    double acc[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = 0.0;
    typename Mma<double>::acc macc = {0.0, 0.0, 0.0, 0.0};
    double bm[4];  // (MMA) this lane's entries of b_I: rows Mma row(lane, q), column lane & 15
    if constexpr (kMma) {
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const int row = 16 * wave + Mma<double>::row(lane, qq), c = lane & 15;
            bm[qq] = load_if(B, (I0 + row) * ldx + c, row < bI && c < nr);
        }
    }

    // T_IJ: rows of block I, columns of block J.  Plain modes: thread (r, q)
    // loads and keeps its own 16 elements.  Transposed modes: it loads 16
    // consecutive elements of factor row J0 + r (tile column r), staged in LDS.
    auto load_tile = [&](int J, T (&dst)[16]) {
        const int64_t J0 = static_cast<int64_t>(J) * SB;
        const int bJ = static_cast<int>((n - J0) < SB ? (n - J0) : SB);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int k = 16 * q + i;
            if (!transposed)
                dst[i] = (r < bI && k < bJ) ? LU[(I0 + r) * ld + J0 + k] : T(0);
            else
                dst[i] = (r < bJ && k < bI) ? LU[(J0 + r) * ld + I0 + k] : T(0);
        }
    };
    const int jfirst = forward ? 0 : nblk - 1, jstep = forward ? 1 : -1;
    T cur[16], nxt[16];
    if (I != jfirst) load_tile(jfirst, nxt);
    for (int J = jfirst; J != I; J += jstep) {
#pragma unroll
        for (int i = 0; i < 16; ++i) cur[i] = nxt[i];
        if (J + jstep != I) load_tile(J + jstep, nxt);
        if (transposed) {
#pragma unroll
            for (int i = 0; i < 16; ++i) Ts[16 * q + i][r] = cur[i];
        } else if (kMma) {
#pragma unroll
            for (int i = 0; i < 16; ++i) Ts[r][16 * q + i] = cur[i];
        }
        const int64_t J0 = static_cast<int64_t>(J) * SB;
        const int bJ = static_cast<int>((n - J0) < SB ? (n - J0) : SB);
        if (wave == 0) {
            double v[NR];
            int spins = 0;
            const bool inl = lane < bJ;
            const double *rowp = X + (J0 + (inl ? lane : 0)) * ldx;
            while (true) {
                // wait on each row's last value (published last, with release),
                // one load a lane a round: the waiting blocks' polls all land
                // on the same few lines, so they are kept few
                bool seen = false;
                poll_value(rowp + (nr - 1), &seen);
                if (__all(seen || !inl)) {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    // then the row's values, every load issued before any is
                    // examined (clamped addresses, no load under a branch)
                    bool ready = true;
#pragma unroll
                    for (int c = 0; c < NR; ++c) {
                        const bool in = inl && c < nr;
                        bool ok;
                        const double pv = poll_value(rowp + (c < nr ? c : 0), &ok);
                        v[c] = in ? pv : 0.0;
                        ready = ready && (ok || !in);
                    }
                    if (__all(ready)) break;
                }
                const bool give_up =
                    (++spins > kSpinLimit) ||
                    __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
                if (__any(give_up)) {
                    if (lane == 0) s_fail = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
#pragma unroll
            for (int c = 0; c < NR; ++c) ys[lane][c] = v[c];
        }
        __syncthreads();
        if (s_fail) break;
        if constexpr (kMma) {
            const int arow = 16 * wave + (lane & 15), bc = lane & 15;
#pragma unroll
            for (int ks = 0; ks < SB / 4; ++ks) {
                const int k = 4 * ks + (lane >> 4);
                const double av = static_cast<double>(Ts[arow][k]);
                const double bv = bc < NR ? ys[k][bc < NR ? bc : 0] : 0.0;
                macc = Mma<double>::step(av, bv, macc);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int k = 16 * q + i;
                const double t = static_cast<double>(transposed ? Ts[r][k] : cur[i]);
#pragma unroll
                for (int c = 0; c < NR; ++c) acc[c] += t * ys[k][c];
            }
        }
        __syncthreads();
    }
    if (s_fail) {
        if (tid == 0) atomicExch(err, 1);  // blocks waiting on this one see it and stop
        return;
    }
    // s = b_I - sum_J T_IJ y_J
    if constexpr (kMma) {
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const int row = 16 * wave + Mma<double>::row(lane, qq), c = lane & 15;
            if (c < NR) ys[row][c < NR ? c : 0] = (row < bI && c < nr) ? bm[qq] - macc[qq] : 0.0;
        }
    } else {
        // reduce the four column quarters of each row
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            acc[c] += __shfl_xor(acc[c], 1);
            acc[c] += __shfl_xor(acc[c], 2);
        }
        if (q == 0) {
#pragma unroll
            for (int c = 0; c < NR; ++c)
                ys[r][c] = (r < bI) ? bval[c] - acc[c] : 0.0;
        }
    }
    __syncthreads();
    // diagonal block: first-solved sub-block f, then the other, g:
    //   x_f = D_f s_f;  s_g -= C x_f;  x_g = D_g s_g
    // (a few right-hand sides: thread t computes entries (i, c) = (e / NR,
    // e mod NR), e = t, t + 256, of the 32 x NR results, each a whole 32-term
    // dot product, no cross-lane reduction: chained shuffles per right-hand
    // side set the pace when the four quarter-rows were reduced that way)
    const int f = forward ? 0 : 1, g = 1 - f;
    if constexpr (kMma) {
        // on the matrix cores: waves 0 and 1 take rows 0 .. 15 and 16 .. 31 of
        // the sub-block, lane & 15 a right-hand side
        const int c = lane & 15, arow = 16 * wave + (lane & 15);
        auto mm = [&](const T (&Mat)[SW][SW + 1], const double (*Vin)[NR]) {
            typename Mma<double>::acc a4 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ks = 0; ks < SW / 4; ++ks) {
                const int k = 4 * ks + (lane >> 4);
                const double av = static_cast<double>(Mat[arow][k]);
                const double bv = c < NR ? Vin[k][c < NR ? c : 0] : 0.0;
                a4 = Mma<double>::step(av, bv, a4);
            }
            return a4;
        };
        if (wave < 2) {
            const auto v = mm(Dd[f], ys + SW * f);
#pragma unroll
            for (int qq = 0; qq < 4; ++qq)
                if (c < NR) xs[SW * f + 16 * wave + Mma<double>::row(lane, qq)][c < NR ? c : 0] = v[qq];
        }
        __syncthreads();
        if (wave < 2) {
            const auto v = mm(Cp, xs + SW * f);
#pragma unroll
            for (int qq = 0; qq < 4; ++qq)
                if (c < NR) ys[SW * g + 16 * wave + Mma<double>::row(lane, qq)][c < NR ? c : 0] -= v[qq];
        }
        __syncthreads();
        if (wave < 2) {
            const auto v = mm(Dd[g], ys + SW * g);
#pragma unroll
            for (int qq = 0; qq < 4; ++qq)
                if (c < NR) xs[SW * g + 16 * wave + Mma<double>::row(lane, qq)][c < NR ? c : 0] = v[qq];
        }
        __syncthreads();
    } else {
        constexpr int NP = (SW * NR + 255) / 256;
#pragma unroll
        for (int pp = 0; pp < NP; ++pp) {
            const int e = tid + 256 * pp;
            if (e < SW * NR) {
                const int i = e / NR, c = e % NR;
                double v = 0.0;
#pragma unroll 8
                for (int j = 0; j < SW; ++j) v += static_cast<double>(Dd[f][i][j]) * ys[SW * f + j][c];
                xs[SW * f + i][c] = v;
            }
        }
        __syncthreads();
#pragma unroll
        for (int pp = 0; pp < NP; ++pp) {
            const int e = tid + 256 * pp;
            if (e < SW * NR) {
                const int i = e / NR, c = e % NR;
                double v = 0.0;
#pragma unroll 8
                for (int j = 0; j < SW; ++j) v += static_cast<double>(Cp[i][j]) * xs[SW * f + j][c];
                ys[SW * g + i][c] -= v;
            }
        }
        __syncthreads();
#pragma unroll
        for (int pp = 0; pp < NP; ++pp) {
            const int e = tid + 256 * pp;
            if (e < SW * NR) {
                const int i = e / NR, c = e % NR;
                double v = 0.0;
#pragma unroll 8
                for (int j = 0; j < SW; ++j) v += static_cast<double>(Dd[g][i][j]) * ys[SW * g + j][c];
                xs[SW * g + i][c] = v;
            }
        }
        __syncthreads();
    }
    // (all right-hand sides store with no branch between the stores: at a
    // branch's join the compiler waits for every store issued before it)
    if (tid < bI) {
        if (nr == NR) {
#pragma unroll
            for (int c = 0; c < NR - 1; ++c) publish_value(X + (I0 + tid) * ldx + c, xs[tid][c]);
            publish_last(X + (I0 + tid) * ldx + NR - 1, xs[tid][NR - 1]);
        } else {
#pragma unroll
            for (int c = 0; c < NR - 1; ++c)
                if (c < nr - 1) publish_value(X + (I0 + tid) * ldx + c, xs[tid][c]);
            publish_last(X + (I0 + tid) * ldx + nr - 1, xs[tid][nr - 1]);
        }
    }
}

// ---------------------------------------------------------------------------
// Single right-hand-side solves with L and U (the refinement and Krylov
// preconditioner): 128-row blocks, half as many block-to-block hand-offs as
// k_trsv, and each diagonal block applied as one product with its FP64
// inverse, computed once after the factorization (k_blkinv128).
constexpr int BI = 128;

// FP64 inverses of the 128 x 128 diagonal blocks of the unit-lower L
// (blockIdx.y = 0) and of the upper U (blockIdx.y = 1), in place in LDS;
// a short last block is padded with the identity.  Output: row I0 + i of
// Linv / Uinv holds row i of block I's inverse (128 columns, zeros included).
//   L: X[i][j] = -(l_ij + sum_{j<k<i} X[i][k] l_kj), columns j from right to
//      left, so column j still holds l_.j while it is read;
//   U: X[j][j] = 1 / u_jj, X[i][j] = -(sum_{i<=k<j} X[i][k] u_kj) / u_jj,
//      columns from left to right.
// Four threads share a row's dot product.
template <typename T>
__global__ __launch_bounds__(512) void k_blkinv128(const T *lu, int64_t ld, int64_t n,
                                                   double *Linv, double *Uinv, double *Wl,
                                                   double *Wu) {
    __shared__ double X[BI][BI + 1];
    __shared__ double Ts[16][BI];
    const int64_t I0 = static_cast<int64_t>(blockIdx.x) * BI;
    const bool upper = blockIdx.y == 1;
    const int bI = static_cast<int>((n - I0) < BI ? (n - I0) : BI);
    const int tid = threadIdx.x;
    {
        T v[BI * BI / 512];  // all loads in flight before the first store
#pragma unroll
        for (int m = 0; m < BI * BI / 512; ++m) {
            const int e = tid + 512 * m, i = e / BI, j = e % BI;
            const bool in = i < bI && j < bI && (upper ? j >= i : j < i);
            v[m] = load_if(lu, (I0 + i) * ld + I0 + j, in);
        }
#pragma unroll
        for (int m = 0; m < BI * BI / 512; ++m) {
            const int e = tid + 512 * m, i = e / BI, j = e % BI;
            const bool in = i < bI && j < bI && (upper ? j >= i : j < i);
            X[i][j] = in ? static_cast<double>(v[m]) : ((i == j && (!upper || i >= bI)) ? 1.0 : 0.0);
        }
    }
    __syncthreads();
    const int i = tid >> 2, h = tid & 3;
    if (!upper) {
        for (int j = BI - 2; j >= 0; --j) {
            double p = 0.0;
            if (i > j)
                for (int k = j + 1 + h; k < i; k += 4) p += X[i][k] * X[k][j];
            p += __shfl_xor(p, 1);
            p += __shfl_xor(p, 2);
            __syncthreads();  // column j has been read everywhere
            if (i > j && h == 0) X[i][j] = -(X[i][j] + p);
            __syncthreads();
        }
    } else {
        for (int j = 0; j < BI; ++j) {
            double p = 0.0;
            if (i < j)
                for (int k = i + h; k < j; k += 4) p += X[i][k] * X[k][j];
            p += __shfl_xor(p, 1);
            p += __shfl_xor(p, 2);
            const double d = X[j][j];
            __syncthreads();  // column j and u_jj have been read everywhere
            if (h == 0) {
                if (i < j) X[i][j] = -p / d;
                else if (i == j) X[j][j] = 1.0 / d;
            }
            __syncthreads();
        }
    }
    double *out = upper ? Uinv : Linv;
    for (int e = tid; e < BI * BI; e += 512) {
        const int r = e / BI, c = e % BI;
        out[(I0 + r) * BI + c] = X[r][c];
    }
    // W = X C, C the coupling of this block with the one solved just before it
    // (L: the tile of block row I, block column I - 1; U: block column I + 1),
    // so the solve can apply x_I = X s' - W y_adjacent once y_adjacent lands.
    // C is staged 16 rows at a time; thread (i, q) forms W[i][32 q .. 32 q + 31].
    const int nblk = static_cast<int>((n + BI - 1) / BI);
    const int Jn = upper ? static_cast<int>(blockIdx.x) + 1 : static_cast<int>(blockIdx.x) - 1;
    if (Jn < 0 || Jn >= nblk) return;  // no such neighbour: W is never read
    const int64_t J0 = static_cast<int64_t>(Jn) * BI;
    const int bJ = static_cast<int>((n - J0) < BI ? (n - J0) : BI);
    const int wi = tid >> 2, wq = tid & 3;
    double wacc[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) wacc[j] = 0.0;
    for (int k0 = 0; k0 < BI; k0 += 16) {
        T v[16 * BI / 512];
#pragma unroll
        for (int m = 0; m < 16 * BI / 512; ++m) {
            const int e = tid + 512 * m, kk = e / BI, j = e % BI;
            v[m] = load_if(lu, (I0 + k0 + kk) * ld + J0 + j, k0 + kk < bI && j < bJ);
        }
#pragma unroll
        for (int m = 0; m < 16 * BI / 512; ++m) {
            const int e = tid + 512 * m;
            Ts[e / BI][e % BI] = static_cast<double>(v[m]);
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < 16; ++kk) {
            const double xk = X[wi][k0 + kk];
#pragma unroll
            for (int j = 0; j < 32; ++j) wacc[j] += xk * Ts[kk][32 * wq + j];
        }
        __syncthreads();
    }
    double *wout = upper ? Wu : Wl;
#pragma unroll
    for (int j = 0; j < 32; ++j) wout[(I0 + wi) * BI + 32 * wq + j] = wacc[j];
}

// Sum of v over each row of 16 lanes, in every lane of the row, by DPP moves
// (register to register): quad permutations [1,0,3,2] and [2,3,0,1], then the
// half-row and row mirrors.  Each step adds a value and its partner's, so all
// lanes of a row end with the same sum.
template <int CTRL>
__device__ inline double dpp_move(double v) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(bits), CTRL, 0xf, 0xf, false);
    const int hi =
        __builtin_amdgcn_update_dpp(0, static_cast<int>(bits >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}
__device__ inline double row16_sum(double v) {
    v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_move<0x141>(v);  // row_half_mirror
    v += dpp_move<0x140>(v);  // row_mirror
    return v;
}

// Eight consecutive factor entries from p (8-element aligned).
template <typename T>
__device__ inline void load_row8(const T *p, T (&dst)[8]) {
    typedef T v4 __attribute__((ext_vector_type(16 / sizeof(T))));
    constexpr int W = 16 / sizeof(T);
#pragma unroll
    for (int c = 0; c < 8 / W; ++c) {
        const v4 v = reinterpret_cast<const v4 *>(p)[c];
#pragma unroll
        for (int e = 0; e < W; ++e) dst[W * c + e] = v[e];
    }
}

// MODE 0: L y = b (forward), MODE 1: U y = b (backward); one right-hand side.
// Same ticket order, mark-as-flag hand-off and bounded waits as k_trsv.
// With D = the block's inverse and W = D C (C its coupling with the adjacent
// block, solved just before it; both from k_blkinv128),
//     x_I = D (b_I - sum_{J not adjacent} T_IJ y_J) - W y_adjacent,
// so everything but the last product is done while the adjacent block is
// still being solved.  Thread (g, c) owns rows RG g .. RG g + RG - 1 of its
// block (RG = 4 in FP32 with 512 threads; 2 in FP64 with 1024 threads and D
// staged in LDS, which keeps the FP64 tiles in registers) and columns
// 8 c .. 8 c + 7 of each coupling tile (prefetched one tile ahead), of D and of
// W, so it reads 8 entries of y_J a tile; a row's 16 partial sums sit in 16
// consecutive lanes and reduce by DPP moves.  Wave 0 polls y_J, one round of
// loads at a time.
template <typename T>
constexpr int trsv128_threads() { return sizeof(T) == 4 ? 512 : 1024; }

template <typename T, int MODE>
__global__ __launch_bounds__(trsv128_threads<T>()) void k_trsv128(const T *LU, int64_t ld,
                                                                  int64_t n, const double *Dinv,
                                                                  const double *W,
                                                                  const double *B, double *X,
                                                                  int64_t ldx, int *sync) {
    constexpr bool forward = MODE == 0;
    constexpr int CG = 8, RG = BI * 16 / trsv128_threads<T>();  // columns, rows a thread owns
    constexpr bool kInvLds = sizeof(T) == 8;
    __shared__ double dl[kInvLds ? BI : 1][BI];
    __shared__ double ys[2][BI];
    __shared__ double ss[BI];
    __shared__ int s_ticket, s_fail;
    int *counter = sync, *err = sync + 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) {
        s_ticket = atomicAdd(counter, 1);
        s_fail = 0;
    }
    __syncthreads();
    const int nblk = static_cast<int>((n + BI - 1) / BI);
    const int I = forward ? s_ticket : nblk - 1 - s_ticket;
    const int64_t I0 = static_cast<int64_t>(I) * BI;
    const int bI = static_cast<int>((n - I0) < BI ? (n - I0) : BI);
    const int g = tid >> 4, c = tid & 15;  // rows RG g .., columns CG c ..
    const int r0 = RG * g, c0 = CG * c;
    if constexpr (kInvLds) {
        constexpr int kPer = BI * BI / trsv128_threads<T>();
        double v[kPer];
#pragma unroll
        for (int m = 0; m < kPer; ++m) v[m] = Dinv[I0 * BI + tid + trsv128_threads<T>() * m];
#pragma unroll
        for (int m = 0; m < kPer; ++m) {
            const int e = tid + trsv128_threads<T>() * m;
            dl[e / BI][e % BI] = v[m];
        }
    }
    double bval[RG];
#pragma unroll
    for (int k = 0; k < RG; ++k) bval[k] = load_if(B, (I0 + r0 + k) * ldx, c == 0 && r0 + k < bI);
    // this thread's part of D: fetched in place of the tile prefetch during
    // the last non-adjacent coupling step (or now, if there is none)
    double dreg[kInvLds ? 1 : RG][CG];
    auto load_dinv = [&]() {
        if constexpr (!kInvLds) {
#pragma unroll
            for (int k = 0; k < RG; ++k)
#pragma unroll
                for (int e = 0; e < CG; ++e) dreg[k][e] = Dinv[(I0 + r0 + k) * BI + c0 + e];
        }
    };
    auto load_tile = [&](int J, T (&dst)[RG][CG]) {
        const int64_t J0 = static_cast<int64_t>(J) * BI;
        const int bJ = static_cast<int>((n - J0) < BI ? (n - J0) : BI);
        if (bI == BI && bJ == BI) {
#pragma unroll
            for (int k = 0; k < RG; ++k) load_row8(LU + (I0 + r0 + k) * ld + J0 + c0, dst[k]);
        } else {
#pragma unroll
            for (int k = 0; k < RG; ++k)
#pragma unroll
                for (int e = 0; e < CG; ++e)
                    dst[k][e] = load_if(LU, (I0 + r0 + k) * ld + J0 + c0 + e,
                                        r0 + k < bI && c0 + e < bJ);
        }
    };
    // Wait for y_J (wave 0, two entries a lane; lanes past the block poll its
    // first entry) and leave it in ys[par] for all threads; false if a wait
    // gave up.  One round of polls at a time: a round left in flight when the
    // wait ends would make a later instruction wait for it (its registers
    // are reused), which measured ~1 us per block on the publication.
    auto await_block = [&](int J, int par) {
        if (wave == 0) {
            const int64_t J0 = static_cast<int64_t>(J) * BI;
            const int bJ = static_cast<int>((n - J0) < BI ? (n - J0) : BI);
            const bool in0 = lane < bJ, in1 = lane + 64 < bJ;
            const double *p0 = X + (J0 + (in0 ? lane : 0)) * ldx;
            const double *p1 = X + (J0 + (in1 ? lane + 64 : 0)) * ldx;
            bool ok0, ok1;
            double v0, v1;
            int spins = 0;
            while (true) {
                v0 = poll_value(p0, &ok0);
                v1 = poll_value(p1, &ok1);
                if (__all(ok0 && ok1)) break;
                const bool give_up =
                    (++spins > kSpinLimit) ||
                    __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
                if (__any(give_up)) {
                    if (lane == 0) s_fail = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            ys[par][lane] = in0 ? v0 : 0.0;
            ys[par][lane + 64] = in1 ? v1 : 0.0;
        }
        __syncthreads();  // (ys[par] is next written two waits later, after another barrier)
        return s_fail == 0;
    };
    const int jfirst = forward ? 0 : nblk - 1, jstep = forward ? 1 : -1;
    const bool has_adj = I != jfirst;
    const int jadj = I - jstep;                       // the adjacent block (through W)
    const bool has_tiles = has_adj && jfirst != jadj;  // other coupling tiles
    T cur[RG][CG], nxt[RG][CG];
    if (has_tiles)
        load_tile(jfirst, nxt);
    else
        load_dinv();
    double acc[RG];
#pragma unroll
    for (int k = 0; k < RG; ++k) acc[k] = 0.0;
    int par = 0;
    bool ok = true;
    if (has_tiles) {
        for (int J = jfirst; J != jadj; J += jstep, par ^= 1) {
#pragma unroll
            for (int k = 0; k < RG; ++k)
#pragma unroll
                for (int e = 0; e < CG; ++e) cur[k][e] = nxt[k][e];
            if (J + jstep != jadj)
                load_tile(J + jstep, nxt);
            else
                load_dinv();
            if (!(ok = await_block(J, par))) break;
            double y[CG];
#pragma unroll
            for (int e = 0; e < CG; ++e) y[e] = ys[par][c0 + e];
#pragma unroll
            for (int k = 0; k < RG; ++k)
#pragma unroll
                for (int e = 0; e < CG; ++e) acc[k] += static_cast<double>(cur[k][e]) * y[e];
        }
    }
    double x[RG];
    if (ok) {
        // x = D (b_I - sum of the non-adjacent couplings)
#pragma unroll
        for (int k = 0; k < RG; ++k) acc[k] = row16_sum(acc[k]);
        if (c == 0) {
#pragma unroll
            for (int k = 0; k < RG; ++k) ss[r0 + k] = (r0 + k < bI) ? bval[k] - acc[k] : 0.0;
        }
        __syncthreads();
        double sv[CG];
#pragma unroll
        for (int e = 0; e < CG; ++e) sv[e] = ss[c0 + e];
#pragma unroll
        for (int k = 0; k < RG; ++k) {
            x[k] = 0.0;
#pragma unroll
            for (int e = 0; e < CG; ++e)
                x[k] += (kInvLds ? dl[r0 + k][c0 + e] : dreg[kInvLds ? 0 : k][e]) * sv[e];
            x[k] = row16_sum(x[k]);
        }
        if (has_adj) {
            // x -= W y_adjacent: W is fetched before the wait
            double wreg[RG][CG];
#pragma unroll
            for (int k = 0; k < RG; ++k)
#pragma unroll
                for (int e = 0; e < CG; ++e) wreg[k][e] = W[(I0 + r0 + k) * BI + c0 + e];
            if ((ok = await_block(jadj, par))) {
                double y[CG];
#pragma unroll
                for (int e = 0; e < CG; ++e) y[e] = ys[par][c0 + e];
#pragma unroll
                for (int k = 0; k < RG; ++k) {
                    double t = 0.0;
#pragma unroll
                    for (int e = 0; e < CG; ++e) t += wreg[k][e] * y[e];
                    x[k] -= row16_sum(t);
                }
            }
        }
    }
    if (!ok) {
        if (tid == 0) atomicExch(err, 1);  // blocks waiting on this one see it and stop
        return;
    }
    // Every lane of a row group holds the group's RG sums (row16_sum leaves a
    // row's total in all 16 lanes), so lane c < RG publishes row r0 + c: one
    // store instruction a wave.
    if (c < RG && r0 + c < bI) {
        double xv = x[0];
#pragma unroll
        for (int k = 1; k < RG; ++k) xv = (c == k) ? x[k] : xv;
        publish_value(X + (I0 + r0 + c) * ldx, xv);
    }
}

// Before a solve: reset the ticket counter and mark every output entry unsolved.
__global__ void k_trsv_prep(double *X, int64_t ldx, int64_t n, int nr, int *sync) {
    if (blockIdx.x == 0 && threadIdx.x == 0) sync[0] = 0;
    const int64_t total = n * nr;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x)
        X[(e / nr) * ldx + e % nr] = __builtin_bit_cast(double, kMark);
}

__device__ inline void atomic_max_nonneg(double *addr, double v) {
    atomicMax(reinterpret_cast<unsigned long long *>(addr),
              static_cast<unsigned long long>(__double_as_longlong(v)));
}

// y = beta y + alpha M x, FP64 accumulation; one wave per two rows.  With
// rowmax != null also the largest row sum of |M| (||M||_inf) into *rowmax,
// from the same reads.
template <typename TM, typename TX, typename TY, int NR>
__global__ __launch_bounds__(256) void k_gemv_n(int64_t rows, int64_t cols, double alpha,
                                                const TM *__restrict__ Mat, int64_t ldm,
                                                const TX *__restrict__ x, int64_t ldx, double beta,
                                                TY *y, int64_t ldy, int nrhs, double *rowmax) {
    const int lane = threadIdx.x & 63;
    const int64_t row0 = (static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6)) * 2;
    if (row0 >= rows) return;
    const bool two = row0 + 1 < rows;
    double a0[NR], a1[NR], s0 = 0.0, s1 = 0.0;
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
        for (int u = 0; u < 4; ++u) {
            s0 += fabs(p0[u]);
            s1 += fabs(p1[u]);
        }
        // (right-hand sides past nrhs read x[0] and accumulate zeros: no
        // load sits under a branch)
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const double xv =
                    static_cast<double>(load_if(x, (c + 64 * u) * ldx + r, r == 0 || r < nrhs));
                a0[r] += p0[u] * xv;
                a1[r] += p1[u] * xv;
            }
    }
    for (; c < cols; c += 64) {
        const double p0 = static_cast<double>(m0[c]), p1 = static_cast<double>(m1[c]);
        s0 += fabs(p0);
        s1 += fabs(p1);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const double xv = static_cast<double>(load_if(x, c * ldx + r, r == 0 || r < nrhs));
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
    if (rowmax != nullptr) {
        for (int off = 32; off > 0; off >>= 1) {
            s0 += __shfl_xor(s0, off);
            s1 += __shfl_xor(s1, off);
        }
        if (lane == 0) atomic_max_nonneg(rowmax, two ? fmax(s0, s1) : s0);
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

// work[chunk][c] = sum over the chunk's 256 rows i of |A[i][c]| (pass 1 of ||A||_1).
__global__ __launch_bounds__(256) void k_colabs_part(int64_t rows, int64_t cols, const double *A,
                                                     int64_t lda, double *work) {
    const int64_t i0 = static_cast<int64_t>(blockIdx.y) * 256;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (c >= cols) return;
    const int64_t i1 = (i0 + 256) < rows ? (i0 + 256) : rows;
    double acc = 0.0;
    for (int64_t i = i0; i < i1; ++i) acc += fabs(A[i * lda + c]);
    work[static_cast<int64_t>(blockIdx.y) * cols + c] = acc;
}

// out[0] = max(out[0], max_c sum_chunks work[chunk][c]).
__global__ void k_colabs_max(int64_t chunks, int64_t cols, const double *work, double *out) {
    double m = 0.0;
    for (int64_t c = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; c < cols;
         c += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        double sum = 0.0;
        for (int64_t k = 0; k < chunks; ++k) sum += work[k * cols + c];
        m = fmax(m, sum);
    }
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) atomic_max_nonneg(out, m);
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

// x[row] = beta x[row] + d[i] with row = scatter ? scatter[i] : i.
template <typename TS>
__global__ void k_axpby_2d(const TS *d, int64_t ldd, double *x, int64_t ldx, int64_t n, int nrhs,
                           double beta, const int *scatter) {
    const int64_t total = n * nrhs;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t i = e / nrhs, r = e % nrhs;
        const double v = static_cast<double>(d[i * ldd + r]);
        double *p = x + (scatter ? static_cast<int64_t>(scatter[i]) : i) * ldx + r;
        *p = (beta == 0.0) ? v : beta * (*p) + v;
    }
}

__global__ void k_fill_f64(double *p, int64_t count, double value) {
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < count;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[e] = value;
}

// ---- Krylov helpers (basis vectors stored contiguously: V[k * n + i]) ----

constexpr int kMdotChunks = 256;  // partial sums per dot product (fixed: deterministic)
constexpr int kMaxBasis = 64;

// part[c * k + j] = sum over chunk c of V_j . w  (chunk c: rows c*cs .. c*cs + cs - 1)
__global__ __launch_bounds__(256) void k_mdot_part(const double *V, int64_t n, int k,
                                                   const double *w, int64_t cs, double *part) {
    __shared__ double red[4];
    const int64_t i0 = static_cast<int64_t>(blockIdx.x) * cs;
    const int64_t i1 = (i0 + cs) < n ? (i0 + cs) : n;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = 0; j < k; ++j) {
        double acc = 0.0;
        for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) acc += V[j * n + i] * w[i];
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (lane == 0) red[wave] = acc;
        __syncthreads();
        if (threadIdx.x == 0)
            part[static_cast<int64_t>(blockIdx.x) * k + j] = (red[0] + red[1]) + (red[2] + red[3]);
        __syncthreads();
    }
}

// h[j] = sum_c part[c * k + j] (+ h[j] when accumulate), in chunk order.
__global__ void k_mdot_sum(const double *part, int chunks, int k, double *h, int accumulate) {
    const int j = threadIdx.x;
    if (j >= k) return;
    double s = 0.0;
    for (int c = 0; c < chunks; ++c) s += part[c * k + j];
    h[j] = accumulate ? h[j] + s : s;
}

// w[i] += sign * sum_j V_j[i] h[j]   (h on the device, k <= kMaxBasis)
__global__ __launch_bounds__(256) void k_lincomb(double *w, int64_t ldw, const double *V, int64_t n,
                                                 int k, const double *h, double sign) {
    __shared__ double hs[kMaxBasis];
    if (threadIdx.x < k) hs[threadIdx.x] = h[threadIdx.x];
    __syncthreads();
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        double s = 0.0;
        for (int j = 0; j < k; ++j) s += V[j * n + i] * hs[j];
        w[i * ldw] += sign * s;
    }
}

// ---- block Krylov helpers: m right-hand sides at once, basis block j stored
// as an n x m row-major matrix at V + j n m (column c of block j is vector j of
// right-hand side c) ----

// part[(chunk k + j) m + c] = sum over the chunk's rows r of V_j[r][c] W[r][c]
// (thread t: column t mod mp, rows t / mp, t / mp + 256 / mp, ...; mp = the
// next power of two >= m, mp <= 64; the partial sums of a column added in a
// fixed order, so the result does not depend on scheduling).
__global__ __launch_bounds__(256) void k_bdot_part(const double *V, int64_t n, int m, int mp,
                                                   int k, const double *W, int64_t ldw,
                                                   int64_t cs, double *part) {
    __shared__ double red[256];
    const int64_t i0 = static_cast<int64_t>(blockIdx.x) * cs;
    const int64_t i1 = (i0 + cs) < n ? (i0 + cs) : n;
    const int c = threadIdx.x & (mp - 1), g = threadIdx.x / mp, ng = 256 / mp;
    for (int j = 0; j < k; ++j) {
        const double *Vj = V + static_cast<int64_t>(j) * n * m;
        double acc = 0.0;
        if (c < m)
            for (int64_t r = i0 + g; r < i1; r += ng) acc += Vj[r * m + c] * W[r * ldw + c];
        red[threadIdx.x] = acc;
        __syncthreads();
        if (threadIdx.x < m) {
            double sum = 0.0;
            for (int q = 0; q < ng; ++q) sum += red[q * mp + threadIdx.x];
            part[(static_cast<int64_t>(blockIdx.x) * k + j) * m + threadIdx.x] = sum;
        }
        __syncthreads();
    }
}

// h[j m + c] = sum_chunk part[(chunk k + j) m + c] (+ h when accumulate), chunk order.
__global__ void k_bdot_sum(const double *part, int chunks, int k, int m, double *h,
                           int accumulate) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= k * m) return;
    double s = 0.0;
    for (int q = 0; q < chunks; ++q) s += part[static_cast<int64_t>(q) * k * m + e];
    h[e] = accumulate ? h[e] + s : s;
}

// W[r][c] += sign * sum_j h[j m + c] V_j[r][c]   (h on the device, k m <= kMaxBasis * 64)
__global__ __launch_bounds__(256) void k_blincomb(double *W, int64_t ldw, const double *V,
                                                  int64_t n, int m, int k, const double *h,
                                                  double sign) {
    __shared__ double hs[kMaxBasis * 64];
    for (int e = threadIdx.x; e < k * m; e += blockDim.x) hs[e] = h[e];
    __syncthreads();
    const int64_t total = n * m;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t r = e / m;
        const int c = static_cast<int>(e - r * m);
        double acc = 0.0;
        for (int j = 0; j < k; ++j) acc += V[static_cast<int64_t>(j) * n * m + e] * hs[j * m + c];
        W[r * ldw + c] += sign * acc;
    }
}

// dst[r][c] = scale[c] * src[r * lds + c]  (dst n x m, ld m; scale on the device)
__global__ void k_bscale(double *dst, const double *src, int64_t lds, int64_t n, int m,
                         const double *scale) {
    const int64_t total = n * m;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t r = e / m;
        const int c = static_cast<int>(e - r * m);
        dst[e] = scale[c] * src[r * lds + c];
    }
}

// dst[i] = alpha * src[i * lds]
__global__ void k_scale_copy(double *dst, const double *src, int64_t lds, int64_t n, double alpha) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        dst[i] = alpha * src[i * lds];
}

// GA = -GB X^T (n x n; GB, X: n x nrhs, nrhs <= K <= 64): the gradient of
// sum(W .* X) with respect to A when X = A^{-1} B and GB = A^{-T} W.  One
// workgroup writes a 32 x 256 tile, one column per thread: the thread keeps
// its row of X in registers (zero past nrhs), the 32 rows of GB sit in LDS
// and are read as broadcasts, and every output row is one coalesced 2 KiB
// store.  Bound: HBM writes of GA (8 n^2 bytes).
template <int K>
__global__ __launch_bounds__(256) void k_grad_a(const double *GB, int64_t ldgb, const double *X,
                                                int64_t ldx, int64_t n, int nrhs, double *GA,
                                                int64_t ldga) {
    constexpr int R = 32;
    __shared__ double gb[R][K];
    const int64_t i0 = static_cast<int64_t>(blockIdx.y) * R;
    const int64_t j = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    for (int e = threadIdx.x; e < R * K; e += 256) {
        const int i = e / K, r = e % K;
        gb[i][r] = load_if(GB, (i0 + i) * ldgb + r, i0 + i < n && r < nrhs);
    }
    double x[K];
#pragma unroll
    for (int r = 0; r < K; ++r) x[r] = load_if(X, j * ldx + r, j < n && r < nrhs);
    __syncthreads();
    if (j >= n) return;
    const int rows = (n - i0) < R ? static_cast<int>(n - i0) : R;
    for (int i = 0; i < rows; ++i) {
        double acc = 0.0;
#pragma unroll
        for (int r = 0; r < K; ++r) acc += gb[i][r] * x[r];
        __builtin_nontemporal_store(-acc, GA + (i0 + i) * ldga + j);  // written once, not reread
    }
}

int grid_for(int64_t total, int threads) {
    int64_t g = (total + threads - 1) / threads;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return static_cast<int>(g);
}

}  // namespace

template <typename T, int MODE>
hipError_t trsv_full_launch(const T *LU, int64_t ld, int64_t n, const T *Dinv, const double *B,
                            double *X, int64_t ldx, int nr, int *sync, hipStream_t s) {
    const int nblk = static_cast<int>((n + SB - 1) / SB);
    hipLaunchKernelGGL(k_trsv_prep, dim3(grid_for(n * nr, 256)), dim3(256), 0, s, X, ldx, n, nr,
                       sync);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (nr <= 1)
        hipLaunchKernelGGL((k_trsv<T, MODE, 1>), dim3(nblk), dim3(256), 0, s, LU, ld, n, Dinv, B, X,
                           ldx, nr, sync);
    else if (nr <= 4)
        hipLaunchKernelGGL((k_trsv<T, MODE, 4>), dim3(nblk), dim3(256), 0, s, LU, ld, n, Dinv, B, X,
                           ldx, nr, sync);
    else if (nr <= 8)
        hipLaunchKernelGGL((k_trsv<T, MODE, 8>), dim3(nblk), dim3(256), 0, s, LU, ld, n, Dinv, B, X,
                           ldx, nr, sync);
    else
        hipLaunchKernelGGL((k_trsv<T, MODE, 16>), dim3(nblk), dim3(256), 0, s, LU, ld, n, Dinv, B,
                           X, ldx, nr, sync);
    return hipGetLastError();
}

template <typename T>
hipError_t trsv_full(int mode, const T *LU, int64_t ld, int64_t n, const T *Dinv, const double *B,
                     double *X, int64_t ldx, int nr, int *sync, hipStream_t s) {
    if (nr < 1 || nr > 16 || n < 1 || B == X) return hipErrorInvalidValue;
    switch (mode) {
    case 0: return trsv_full_launch<T, 0>(LU, ld, n, Dinv, B, X, ldx, nr, sync, s);
    case 1: return trsv_full_launch<T, 1>(LU, ld, n, Dinv, B, X, ldx, nr, sync, s);
    case 2: return trsv_full_launch<T, 2>(LU, ld, n, Dinv, B, X, ldx, nr, sync, s);
    case 3: return trsv_full_launch<T, 3>(LU, ld, n, Dinv, B, X, ldx, nr, sync, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t block_inverses128(const T *lu, int64_t ld, int64_t n, double *Linv, double *Uinv,
                             double *Wl, double *Wu, hipStream_t s) {
    if (n < 1) return hipSuccess;
    const unsigned nblk = static_cast<unsigned>((n + BI - 1) / BI);
    hipLaunchKernelGGL(k_blkinv128<T>, dim3(nblk, 2), dim3(512), 0, s, lu, ld, n, Linv, Uinv, Wl,
                       Wu);
    return hipGetLastError();
}

template <typename T>
hipError_t trsv128(int mode, const T *LU, int64_t ld, int64_t n, const double *Dinv,
                   const double *W, const double *B, double *X, int64_t ldx, int *sync,
                   hipStream_t s) {
    if (n < 1 || B == X || (mode != 0 && mode != 1)) return hipErrorInvalidValue;
    const int nblk = static_cast<int>((n + BI - 1) / BI);
    hipLaunchKernelGGL(k_trsv_prep, dim3(grid_for(n, 256)), dim3(256), 0, s, X, ldx, n, 1, sync);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned threads = trsv128_threads<T>();
    if (mode == 0)
        hipLaunchKernelGGL((k_trsv128<T, 0>), dim3(nblk), dim3(threads), 0, s, LU, ld, n, Dinv, W,
                           B, X, ldx, sync);
    else
        hipLaunchKernelGGL((k_trsv128<T, 1>), dim3(nblk), dim3(threads), 0, s, LU, ld, n, Dinv, W,
                           B, X, ldx, sync);
    return hipGetLastError();
}

template <typename TM, typename TX, typename TY>
hipError_t gemv_n(int64_t rows, int64_t cols, double alpha, const TM *Mat, int64_t ldm,
                  const TX *x, int64_t ldx, double beta, TY *y, int64_t ldy, int nrhs,
                  hipStream_t s, double *rowmax) {
    if (rows <= 0 || nrhs <= 0) return hipSuccess;
    if (nrhs > 16 || (rowmax != nullptr && nrhs > 4)) return hipErrorInvalidValue;
    const int64_t grid = (rows + 7) / 8;
    if (nrhs == 1)
        hipLaunchKernelGGL((k_gemv_n<TM, TX, TY, 1>), dim3(static_cast<unsigned>(grid)), dim3(256),
                           0, s, rows, cols, alpha, Mat, ldm, x, ldx, beta, y, ldy, nrhs, rowmax);
    else if (nrhs <= 4)
        hipLaunchKernelGGL((k_gemv_n<TM, TX, TY, 4>), dim3(static_cast<unsigned>(grid)), dim3(256),
                           0, s, rows, cols, alpha, Mat, ldm, x, ldx, beta, y, ldy, nrhs, rowmax);
    else if constexpr (sizeof(TX) == 8 && sizeof(TY) == 8)  // FP64 vectors: matrix cores
        return gemm_skinny<TM>(rows, cols, alpha, Mat, ldm, reinterpret_cast<const double *>(x),
                               ldx, beta, reinterpret_cast<double *>(y), ldy, nrhs, s);
    else
        hipLaunchKernelGGL((k_gemv_n<TM, TX, TY, 16>), dim3(static_cast<unsigned>(grid)),
                           dim3(256), 0, s, rows, cols, alpha, Mat, ldm, x, ldx, beta, y, ldy,
                           nrhs, nullptr);
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
                    double beta, hipStream_t s, const int *scatter) {
    if (n <= 0 || nrhs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_axpby_2d<TS>, dim3(grid_for(n * nrhs, 256)), dim3(256), 0, s, d, ldd, x,
                       ldx, n, nrhs, beta, scatter);
    return hipGetLastError();
}

hipError_t norm_one(const double *A, int64_t lda, int64_t n, double *work, double *out,
                    hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t chunks = (n + 255) / 256;
    dim3 grid(static_cast<unsigned>((n + 255) / 256), static_cast<unsigned>(chunks));
    hipLaunchKernelGGL(k_colabs_part, grid, dim3(256), 0, s, n, n, A, lda, work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_colabs_max, dim3(grid_for(n, 256)), dim3(256), 0, s, chunks, n, work,
                       out);
    return hipGetLastError();
}

// y = beta y + H x for one right-hand side, H held transposed as BF16 bit
// patterns (Ht[k][i] = H[i][k], row pitch ldk, zero past column n): the
// multiplier of the split-BF16 path, exact in BF16, read at half the bytes
// of its FP32 copy.  FP64 accumulation.  Pass 1: workgroup (ib, kb) takes
// rows k of one block of Ht (kbsize of them) for 2048 consecutive i, eight a
// thread (one 16-byte load a row), into part[kb][i]; pass 2 adds the blocks
// in order, so the result does not depend on scheduling.
constexpr int kHtMaxKB = 4096;

__global__ __launch_bounds__(256) void k_gemv_ht_part(int64_t n, const uint16_t *__restrict__ Ht,
                                                      int64_t ldk, const double *__restrict__ x,
                                                      int64_t ldx, int kbsize, double *part) {
    __shared__ double xs[kHtMaxKB];
    const int64_t i0 = static_cast<int64_t>(blockIdx.x) * 2048 + 8 * threadIdx.x;
    const int64_t k0 = static_cast<int64_t>(blockIdx.y) * kbsize;
    const int kc = static_cast<int>((n - k0) < kbsize ? (n - k0) : kbsize);
    for (int t = threadIdx.x; t < kc; t += 256) xs[t] = x[(k0 + t) * ldx];
    __syncthreads();
    if (i0 >= n) return;
    double acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = 0.0;
    const uint16_t *p = Ht + k0 * ldk + i0;
#pragma unroll 4
    for (int t = 0; t < kc; ++t) {
        const uint4 v = *reinterpret_cast<const uint4 *>(p + t * ldk);
        const double xv = xs[t];
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            acc[2 * q] += static_cast<double>(__uint_as_float(w[q] << 16)) * xv;
            acc[2 * q + 1] += static_cast<double>(__uint_as_float(w[q] & 0xffff0000u)) * xv;
        }
    }
    double *o = part + static_cast<int64_t>(blockIdx.y) * n + i0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
        if (i0 + u < n) o[u] = acc[u];
}

__global__ __launch_bounds__(256) void k_gemv_ht_sum(int64_t n, int nkb,
                                                     const double *__restrict__ part, double beta,
                                                     double *y, int64_t ldy) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int kb = 0; kb < nkb; ++kb) s += part[kb * n + i];
    y[i * ldy] = beta == 0.0 ? s : beta * y[i * ldy] + s;
}

int64_t gemv_ht_blocks(int64_t n) {
    int64_t kb = (n + 63) / 64;
    if (kb < 256) kb = 256;
    if (kb > kHtMaxKB) kb = kHtMaxKB;
    return (n + kb - 1) / kb;
}

hipError_t gemv_ht(int64_t n, const uint16_t *Ht, int64_t ldk, const double *x, int64_t ldx,
                   double beta, double *y, int64_t ldy, double *part, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (ldk % 8 != 0 || ldk < (n + 7) / 8 * 8) return hipErrorInvalidValue;
    const int64_t nkb = gemv_ht_blocks(n), kbsize = (n + nkb - 1) / nkb;
    const int64_t nib = (n + 2047) / 2048;
    if (nib > 65535 || nkb > 65535 || kbsize > kHtMaxKB) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gemv_ht_part, dim3(static_cast<unsigned>(nib), static_cast<unsigned>(nkb)),
                       dim3(256), 0, s, n, Ht, ldk, x, ldx, static_cast<int>(kbsize), part);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gemv_ht_sum, dim3(grid_for(n, 256)), dim3(256), 0, s, n,
                       static_cast<int>(nkb), part, beta, y, ldy);
    return hipGetLastError();
}

hipError_t fill_f64(double *p, int64_t count, double value, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(count, 256)), dim3(256), 0, s, p, count, value);
    return hipGetLastError();
}

hipError_t mdot(const double *V, int64_t n, int k, const double *w, double *part, double *h,
                bool accumulate, hipStream_t s) {
    if (k < 1 || k > kMaxBasis || n < 1) return hipErrorInvalidValue;
    const int64_t cs = ((n + kMdotChunks - 1) / kMdotChunks + 255) / 256 * 256;
    const int chunks = static_cast<int>((n + cs - 1) / cs);
    hipLaunchKernelGGL(k_mdot_part, dim3(chunks), dim3(256), 0, s, V, n, k, w, cs, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mdot_sum, dim3(1), dim3(kMaxBasis), 0, s, part, chunks, k, h,
                       accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t lincomb(double *w, int64_t ldw, const double *V, int64_t n, int k, const double *h,
                   double sign, hipStream_t s) {
    if (k < 1 || k > kMaxBasis || n < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_lincomb, dim3(grid_for(n, 256)), dim3(256), 0, s, w, ldw, V, n, k, h,
                       sign);
    return hipGetLastError();
}

hipError_t bdot(const double *V, int64_t n, int m, int k, const double *W, int64_t ldw,
                double *part, double *h, bool accumulate, hipStream_t s) {
    if (k < 1 || k > kMaxBasis || n < 1 || m < 1 || m > 64) return hipErrorInvalidValue;
    int mp = 1;
    while (mp < m) mp <<= 1;
    const int64_t chunks = (n + 255) / 256 < kMdotChunks ? (n + 255) / 256 : kMdotChunks;
    const int64_t cs = (n + chunks - 1) / chunks;
    hipLaunchKernelGGL(k_bdot_part, dim3(static_cast<unsigned>(chunks)), dim3(256), 0, s, V, n, m,
                       mp, k, W, ldw, cs, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bdot_sum, dim3((k * m + 255) / 256), dim3(256), 0, s, part,
                       static_cast<int>(chunks), k, m, h, accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t blincomb(double *W, int64_t ldw, const double *V, int64_t n, int m, int k,
                    const double *h, double sign, hipStream_t s) {
    if (k < 1 || k > kMaxBasis || n < 1 || m < 1 || m > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_blincomb, dim3(grid_for(n * m, 256)), dim3(256), 0, s, W, ldw, V, n, m, k,
                       h, sign);
    return hipGetLastError();
}

hipError_t bscale(double *dst, const double *src, int64_t lds, int64_t n, int m,
                  const double *scale, hipStream_t s) {
    if (n < 1 || m < 1) return hipSuccess;
    hipLaunchKernelGGL(k_bscale, dim3(grid_for(n * m, 256)), dim3(256), 0, s, dst, src, lds, n, m,
                       scale);
    return hipGetLastError();
}

hipError_t scale_copy(double *dst, const double *src, int64_t lds, int64_t n, double alpha,
                      hipStream_t s) {
    if (n < 1) return hipSuccess;
    hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(n, 256)), dim3(256), 0, s, dst, src, lds, n,
                       alpha);
    return hipGetLastError();
}

hipError_t grad_a(const double *GB, int64_t ldgb, const double *X, int64_t ldx, int64_t n,
                  int nrhs, double *GA, int64_t ldga, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (nrhs < 1 || nrhs > 64) return hipErrorInvalidValue;
    dim3 grid(static_cast<unsigned>((n + 255) / 256), static_cast<unsigned>((n + 31) / 32));
    if (grid.y > 65535u) return hipErrorInvalidValue;
    if (nrhs <= 16)
        hipLaunchKernelGGL(k_grad_a<16>, grid, dim3(256), 0, s, GB, ldgb, X, ldx, n, nrhs, GA, ldga);
    else if (nrhs <= 32)
        hipLaunchKernelGGL(k_grad_a<32>, grid, dim3(256), 0, s, GB, ldgb, X, ldx, n, nrhs, GA, ldga);
    else
        hipLaunchKernelGGL(k_grad_a<64>, grid, dim3(256), 0, s, GB, ldgb, X, ldx, n, nrhs, GA, ldga);
    return hipGetLastError();
}

template hipError_t block_inverses128<double>(const double *, int64_t, int64_t, double *,
                                              double *, double *, double *, hipStream_t);
template hipError_t block_inverses128<float>(const float *, int64_t, int64_t, double *, double *,
                                             double *, double *, hipStream_t);
template hipError_t trsv128<double>(int, const double *, int64_t, int64_t, const double *,
                                    const double *, const double *, double *, int64_t, int *,
                                    hipStream_t);
template hipError_t trsv128<float>(int, const float *, int64_t, int64_t, const double *,
                                   const double *, const double *, double *, int64_t, int *,
                                   hipStream_t);
template hipError_t trsv_full<double>(int, const double *, int64_t, int64_t, const double *,
                                      const double *, double *, int64_t, int, int *, hipStream_t);
template hipError_t trsv_full<float>(int, const float *, int64_t, int64_t, const float *,
                                     const double *, double *, int64_t, int, int *, hipStream_t);
template hipError_t gemv_n<double, double, double>(int64_t, int64_t, double, const double *,
                                                   int64_t, const double *, int64_t, double,
                                                   double *, int64_t, int, hipStream_t, double *);
template hipError_t gemv_n<float, float, double>(int64_t, int64_t, double, const float *, int64_t,
                                                 const float *, int64_t, double, double *, int64_t,
                                                 int, hipStream_t, double *);
template hipError_t gemv_n<float, double, double>(int64_t, int64_t, double, const float *,
                                                  int64_t, const double *, int64_t, double,
                                                  double *, int64_t, int, hipStream_t, double *);
template hipError_t gemv_t<double, double, double>(int64_t, int64_t, const double *, int64_t,
                                                   const double *, int64_t, double *, int64_t, int,
                                                   double *, hipStream_t);
template hipError_t gemv_t<float, double, float>(int64_t, int64_t, const float *, int64_t,
                                                 const double *, int64_t, float *, int64_t, int,
                                                 double *, hipStream_t);
template hipError_t gemv_t<float, double, double>(int64_t, int64_t, const float *, int64_t,
                                                  const double *, int64_t, double *, int64_t, int,
                                                  double *, hipStream_t);
template hipError_t axpby_2d<double>(const double *, int64_t, double *, int64_t, int64_t, int,
                                     double, hipStream_t, const int *);
template hipError_t axpby_2d<float>(const float *, int64_t, double *, int64_t, int64_t, int, double,
                                    hipStream_t, const int *);

}  // namespace rmge
