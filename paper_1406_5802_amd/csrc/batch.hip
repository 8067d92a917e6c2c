// Many independent systems of uneven order solved by the method in one
// device-resident pass: per system s, the multiplier H_s (dense Gaussian or
// circulant with a Gaussian first column; Definition defrndm, Section 6),
// M_s = A_s H_s (Fact faprepr), block Gaussian elimination with no pivoting in
// FP32 (eq. eqgenp with pivot blocks of nb_s columns), and FP64 refinement of
// x_s = H_s U_s^{-1} L_s^{-1} b_s by restarted flexible GMRES preconditioned
// with the factors (the Section 8.1 refinement, with a Krylov inner solver).
//
// Launch chain (all on one stream, no host synchronisation, no allocation, so
// it can be captured once into a HIP graph and replayed):
//   k_batch_reset           tickets and per-system status
//   batch_normals           every multiplier's random parameters
//   batch_fft_spectra       circulants: period-m kernel and its half spectrum
//   batch_gemm_f32          Gaussian products, 64 x 64 tiles of all systems
//   batch_fft_rows          circulant products, one row a workgroup
//   k_batch_factor          one workgroup per system, largest first (ticket)
//   k_batch_refine          one workgroup per system, largest first (ticket)
//   k_batch_mark_fallback   the systems still above tol are marked, then
//   batch_gemm_f64,         their FP64 products over the whole device,
//   batch_fft_rows<double>
//   k_batch_factor64        FP64 GENP and refinement, one workgroup per
//   k_batch_refine64        marked system, largest first (ticket)
// The factor and refinement kernels are persistent: a grid of a few
// workgroups per compute unit takes systems from a device ticket counter in
// descending order of size until the queue is empty, so the large systems
// start first and the small ones fill the tail.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/rmge.h"
#include "mfma.h"
#include "rmge_impl.h"

namespace rmge {
namespace {

constexpr int kBatchMaxN = 1024;
constexpr int kBatchThreads = 256;
constexpr int kBatchMaxRestart = 32;

// One system in queue order (largest first).
struct BatchDesc {
    int n, kind, nb, sys;  // order, multiplier kind, panel width, index in the caller's list
    int64_t a_off, v_off;  // A_s (n x n, ld n) and b_s, x_s (n) in the caller's buffers
    int64_t m_off;         // factors (FP32, n x n) in the LU pool
    int64_t g_off;         // Gaussian: G (FP32 n x n) in the G pool; circulant: c (FP64 n)
    int64_t k_off;         // Krylov workspace (FP64) in the K pool
};

// Per-system results, indexed by the caller's order.
struct BatchOut {
    int *status;  // RMGE_OK, RMGE_ZERO_PIVOT, RMGE_NONFINITE, RMGE_NOT_CONVERGED
    int *iters;   // inner GMRES iterations
    double *eta;  // final normwise backward error
    double *eta0; // backward error of the unrefined solution
    int64_t *info;  // index of the first zero or non-finite pivot, -1 if none
    int *fp64;      // 1 if the system was solved again from FP64 factors
    int *tickets;   // [0] refinement, [1 + k] factorization of size bucket k, [6] fallback
};

__global__ void k_batch_reset(int count, BatchOut out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 8) out.tickets[i] = 0;
    if (i < count) {
        out.status[i] = RMGE_OK;
        out.iters[i] = 0;
        out.eta[i] = 0.0;
        out.eta0[i] = 0.0;
        out.info[i] = -1;
        out.fp64[i] = 0;
    }
}

// Lane `src`'s value of x, in every lane (v_readlane; src wave-uniform).
__device__ inline float lane_value(float x, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), src));
}
__device__ inline double lane_value(double x, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), src);
    return __hiloint2double(hi, lo);
}

// ------------------------------------------------------------------ factor
//
// GENP of one n x n FP32 matrix (row-major, ld n) by one workgroup, in place:
// for each pivot block of b <= NB columns at k0,
//   (a) wave 0 factors the b x b diagonal block B = L11 U11 in registers
//       (lane i holds row i; the pivot row reaches the other lanes by
//       readlane) and leaves it, with the pivots' reciprocals, in LDS;
//   (b) U12 = L11^{-1} A12 (one thread a column) and L21 = A21 U11^{-1} (one
//       thread a row) by substitution, 16 unknowns at a time in registers:
//       the earlier ones' contributions are taken out first, then the 16 are
//       solved in place (substitution, unlike products with explicit
//       inverses, keeps the solves backward stable whatever the condition of
//       L11 and U11);
//   (d) A22 -= L21 U12 on the FP32 matrix cores: each wave takes 32-row bands,
//       keeps the band's L21 fragments in registers and sweeps U12 64 columns
//       at a time (all of a round's reads in flight together), updating A22
//       in place.
// These are eq. eqgenp's B^{-1} C and D B^{-1} with B factored, and its Schur
// update; a zero or non-finite pivot stops the system with its status and
// index (the pivots' reciprocals multiply, as in the single-system kernels).
// T = float for the batch's factors, double for the FP64 fallback.
template <int NB, typename T>
__device__ void factor_diag(T *a, int n, int k0, int b, int *status, int64_t *info, T *sd,
                            T *sinv, int *sflag) {
    constexpr int LDD = NB + 1;
    const int lane = threadIdx.x & 63;
    T r[NB];
    const bool in = lane < b;
    const T *row = a + static_cast<int64_t>(k0 + (in ? lane : 0)) * n + k0;
#pragma unroll
    for (int c = 0; c < NB; ++c) r[c] = (c < b && in) ? row[c] : T(0);
    int fail = 0;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if (j < b && fail == 0) {
            const T p = lane_value(r[j], j);
            if (p == T(0) || !isfinite(p)) {
                fail = (p == T(0)) ? RMGE_ZERO_PIVOT : RMGE_NONFINITE;
                if (lane == 0) {
                    *status = fail;
                    *info = k0 + j;
                }
            } else {
                const T inv = T(1) / p;
                if (lane > j) r[j] *= inv;
#pragma unroll
                for (int c = j + 1; c < NB; ++c) {
                    const T u = lane_value(r[c], j);
                    if (lane > j) r[c] -= r[j] * u;
                }
            }
        }
    }
    if (lane == 0) *sflag = fail;
    if (fail || !in) return;
    T dg = T(1);
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        if (c == lane) dg = r[c];
        if (c < b) {
            sd[lane * LDD + c] = r[c];
            a[static_cast<int64_t>(k0 + lane) * n + k0 + c] = r[c];
        }
    }
    sinv[lane] = T(1) / dg;
}

// x <- L11^{-1} x for one column (stride n) of the block row: b unknowns, 16 a
// round in registers.
template <int NB, typename T>
__device__ inline void solve_col(T *col, int n, int b, const T *sd) {
    constexpr int LDD = NB + 1;
    for (int s0 = 0; s0 < b; s0 += 16) {
        T x[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) x[i] = load_if(col, static_cast<int64_t>(s0 + i) * n, s0 + i < b);
        // earlier unknowns, already final in memory: sixteen reads in flight
        // at a time, applied in ascending order
        for (int j0 = 0; j0 < s0; j0 += 16) {
            T u[16];
#pragma unroll
            for (int t = 0; t < 16; ++t) u[t] = col[static_cast<int64_t>(j0 + t) * n];
#pragma unroll
            for (int t = 0; t < 16; ++t)
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    x[i] -= sd[(s0 + i < b ? s0 + i : 0) * LDD + j0 + t] * u[t];
        }
#pragma unroll
        for (int i = 1; i < 16; ++i)
#pragma unroll
            for (int j = 0; j < i; ++j) x[i] -= sd[(s0 + i < b ? s0 + i : 0) * LDD + s0 + j] * x[j];
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (s0 + i < b) col[static_cast<int64_t>(s0 + i) * n] = x[i];
    }
}

// y <- y U11^{-1} for one row of the block column: b unknowns, 16 a round.
template <int NB, typename T>
__device__ inline void solve_row(T *row, int b, const T *sd, const T *sinv) {
    constexpr int LDD = NB + 1;
    for (int s0 = 0; s0 < b; s0 += 16) {
        T y[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) y[j] = load_if(row, s0 + j, s0 + j < b);
        for (int i0 = 0; i0 < s0; i0 += 16) {
            T v[16];
#pragma unroll
            for (int t = 0; t < 16; ++t) v[t] = row[i0 + t];
#pragma unroll
            for (int t = 0; t < 16; ++t)
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    y[j] -= v[t] * sd[(i0 + t) * LDD + (s0 + j < b ? s0 + j : 0)];
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) {
#pragma unroll
            for (int i = 0; i < j; ++i) y[j] -= y[i] * sd[(s0 + i) * LDD + (s0 + j < b ? s0 + j : 0)];
            y[j] *= sinv[s0 + j < b ? s0 + j : 0];
        }
#pragma unroll
        for (int j = 0; j < 16; ++j)
            if (s0 + j < b) row[s0 + j] = y[j];
    }
}

template <int NB, typename T>
__device__ void factor_system(T *a, int n, int *status, int64_t *info, T *sd, T *sinv,
                              int *sflag) {
    using acc_t = typename Mma<T>::acc;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int KS = NB / 4;
    for (int k0 = 0; k0 < n; k0 += NB) {
        const int b = min(NB, n - k0);
        if (wave == 0) factor_diag<NB, T>(a, n, k0, b, status, info, sd, sinv, sflag);
        __syncthreads();
        if (*sflag != 0) return;
        const int r0 = k0 + b, rest = n - r0;
        if (rest <= 0) break;
        // (b) U12 columns, then L21 rows
        for (int w = tid; w < 2 * rest; w += kBatchThreads) {
            if (w < rest)
                solve_col<NB, T>(a + static_cast<int64_t>(k0) * n + r0 + w, n, b, sd);
            else
                solve_row<NB, T>(a + static_cast<int64_t>(r0 + w - rest) * n + k0, b, sd, sinv);
        }
        __syncthreads();
        // (d) A22 -= L21 U12, 32-row bands by wave, 32-column tiles
        const int bands = (rest + 31) / 32;
        for (int band = wave; band < bands; band += kBatchThreads / 64) {
            const int rb = r0 + 32 * band;
            T af[2][KS];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi) {
                const int row = rb + 16 * bi + (lane & 15);
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    const int k = 4 * ks + (lane >> 4);
                    af[bi][ks] = -load_if(a, static_cast<int64_t>(row) * n + k0 + k,
                                          row < n && k < b);
                }
            }
            // CT 16-column tiles a round: all of the round's C and U12 reads
            // are issued before its multiply-adds (CT = 4 measured against 2:
            // FP32 factorisations 33.1 against 35.6 ms, FP64 fallback 55.7
            // against 67.9 ms for the 4096-system batch)
            constexpr int CT = 4;
            for (int cb = r0; cb < n; cb += 16 * CT) {
                acc_t acc[2][CT];
                T bf[KS][CT];
#pragma unroll
                for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                    for (int bj = 0; bj < CT; ++bj)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int row = rb + 16 * bi + Mma<T>::row(lane, q);
                            const int col = cb + 16 * bj + (lane & 15);
                            acc[bi][bj][q] = load_if(a, static_cast<int64_t>(row) * n + col,
                                                     row < n && col < n);
                        }
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    const int k = 4 * ks + (lane >> 4);
#pragma unroll
                    for (int bj = 0; bj < CT; ++bj) {
                        const int col = cb + 16 * bj + (lane & 15);
                        bf[ks][bj] = load_if(a, static_cast<int64_t>(k0 + k) * n + col,
                                             k < b && col < n);
                    }
                }
#pragma unroll
                for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                        for (int bj = 0; bj < CT; ++bj)
                            acc[bi][bj] = Mma<T>::step(af[bi][ks], bf[ks][bj], acc[bi][bj]);
#pragma unroll
                for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                    for (int bj = 0; bj < CT; ++bj)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int row = rb + 16 * bi + Mma<T>::row(lane, q);
                            const int col = cb + 16 * bj + (lane & 15);
                            if (row < n && col < n)
                                a[static_cast<int64_t>(row) * n + col] = acc[bi][bj][q];
                        }
            }
        }
        __syncthreads();
    }
}

// One size bucket's systems (a contiguous range of the queue, all with pivot
// blocks of NB columns), taken in order from the bucket's ticket counter.
template <int NB>
__global__ __launch_bounds__(kBatchThreads) void k_batch_factor(int count,
                                                                 const BatchDesc *__restrict__ d,
                                                                 float *lu_pool, BatchOut out,
                                                                 int *ticket) {
    __shared__ float sd[NB * (NB + 1)], sinv[NB];
    __shared__ int sflag, sq;
    while (true) {
        if (threadIdx.x == 0) sq = atomicAdd(ticket, 1);
        __syncthreads();
        const int q = sq;
        __syncthreads();
        if (q >= count) return;
        const BatchDesc s = d[q];
        factor_system<NB, float>(lu_pool + s.m_off, s.n, out.status + s.sys, out.info + s.sys, sd,
                                 sinv, &sflag);
        __syncthreads();
    }
}

// -------------------------------------------------------------- refinement
//
// Workgroup-wide pieces of one system's solve, called by all 256 threads.
// Vectors of the system live in LDS (FP64, n <= 1024); matrices are read from
// global memory: A in FP64 (the caller's), the factors and a Gaussian G in
// FP32, a circulant's first column in LDS.

struct RefineParams {
    int restart, max_iters;
    double tol;
    // > 0: after four iterations of a cycle, stop a system whose residual,
    // reduced at the cycle's mean rate so far, would need more than giveup x
    // max_iters iterations in all (it is left not converged, for the FP64
    // stage after it); 0: never
    double giveup;
};

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}

// Sum (or max) of one value per thread over the workgroup; every thread gets it.
__device__ inline double block_reduce(double v, bool is_max, double *red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = is_max ? wave_max(v) : wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int w = 1; w < kBatchThreads / 64; ++w) r = is_max ? fmax(r, red[w]) : r + red[w];
    return r;
}

// y = M x for an n x n row-major M (FP64 or FP32, ld n), x and y in LDS: each
// wave takes eight rows at a time, its lanes consecutive columns, two 64-column
// chunks a round, so sixteen loads a lane are in flight (a single workgroup
// streams its system's matrix: its loads in flight set the bandwidth it gets).
// With rowsum != null, also the largest row sum of |M| into *rowsum (thread
// 0's copy is the result).
template <typename TM>
__device__ __attribute__((always_inline)) inline void block_matvec(const TM *__restrict__ M, int n, const double *x, double *y,
                             double *rowsum, double *red) {
    constexpr int RW = 8;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int NW = kBatchThreads / 64;
    double worst = 0.0;
    for (int r0 = RW * wave; r0 < n; r0 += RW * NW) {
        double acc[RW], asum[RW];
#pragma unroll
        for (int u = 0; u < RW; ++u) acc[u] = asum[u] = 0.0;
        for (int c0 = 0; c0 < n; c0 += 128) {
            const int c1 = c0 + lane, c2 = c0 + 64 + lane;
            const double x1 = c1 < n ? x[c1] : 0.0, x2 = c2 < n ? x[c2] : 0.0;
            TM m1[RW], m2[RW];
#pragma unroll
            for (int u = 0; u < RW; ++u) {
                const int r = r0 + u;
                const int64_t base = static_cast<int64_t>(r) * n;
                m1[u] = load_if(M, base + c1, r < n && c1 < n);
                m2[u] = load_if(M, base + c2, r < n && c2 < n);
            }
#pragma unroll
            for (int u = 0; u < RW; ++u) {
                const double a1 = static_cast<double>(m1[u]), a2 = static_cast<double>(m2[u]);
                acc[u] += a1 * x1;
                acc[u] += a2 * x2;
                asum[u] += fabs(a1);
                asum[u] += fabs(a2);
            }
        }
#pragma unroll
        for (int u = 0; u < RW; ++u) {
            const double v = wave_sum(acc[u]);
            if (rowsum) worst = fmax(worst, wave_sum(asum[u]));
            if (lane == 0 && r0 + u < n) y[r0 + u] = v;
        }
    }
    if (rowsum) {
        const double w = block_reduce(worst, true, red);
        if (threadIdx.x == 0) *rowsum = w;
    }
    __syncthreads();
}

// y <- L^{-1} y (unit lower) or U^{-1} y (upper) with the packed factors
// (FP32, or FP64 for the fallback) at lu (ld n), y in LDS (FP64): BLK-row
// diagonal blocks solved by wave 0 in registers (each lane one row, the solved
// values passed by readlane), the coupling to the rows not yet solved taken
// out by all threads.
template <bool UPPER, typename TF>
__device__ void block_trsv(const TF *__restrict__ lu, int n, double *y) {
    constexpr int BLK = 32;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nblk = (n + BLK - 1) / BLK;
    for (int t = 0; t < nblk; ++t) {
        const int blk = UPPER ? nblk - 1 - t : t;
        const int b0 = BLK * blk, bs = min(BLK, n - b0);
        if (wave == 0) {
            const bool in = lane < bs;
            const int row = b0 + (in ? lane : 0);
            TF lr[BLK];
            const TF *lp = lu + static_cast<int64_t>(row) * n + b0;
#pragma unroll
            for (int j = 0; j < BLK; ++j) lr[j] = (j < bs && in) ? lp[j] : TF(0);
            double yi = in ? y[b0 + lane] : 0.0;
            if (UPPER) {
                double dinv = 1.0;
#pragma unroll
                for (int j = 0; j < BLK; ++j)
                    if (j == lane) dinv = 1.0 / static_cast<double>(lr[j]);
#pragma unroll
                for (int j = BLK - 1; j >= 0; --j) {
                    if (j < bs) {
                        if (lane == j) yi *= dinv;
                        const double yj = lane_value(yi, j);
                        if (lane < j) yi -= static_cast<double>(lr[j]) * yj;
                    }
                }
            } else {
#pragma unroll
                for (int j = 0; j < BLK; ++j) {
                    if (j < bs) {
                        const double yj = lane_value(yi, j);
                        if (lane > j) yi -= static_cast<double>(lr[j]) * yj;
                    }
                }
            }
            if (in) y[b0 + lane] = yi;
        }
        __syncthreads();
        // the rows not yet solved lose the block's contribution: 16 lanes a row
        // (lane `sub` takes columns sub and sub + 16 of the block, so a row's
        // 32 values are read by consecutive lanes), four rows a wave at a time
        // and four such groups in flight, the row sums by shuffles in the group
        const int rlo = UPPER ? 0 : b0 + bs, rhi = UPPER ? b0 : n;
        const int sub = lane & 15, grp = lane >> 4;
        const double y1 = sub < bs ? y[b0 + sub] : 0.0;
        const double y2 = sub + 16 < bs ? y[b0 + sub + 16] : 0.0;
        for (int base = rlo + 16 * wave; base < rhi; base += 16 * (kBatchThreads / 64)) {
            double acc[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int r = base + 4 * k + grp;
                const bool in = r < rhi;
                const TF *l1 = lu + static_cast<int64_t>(in ? r : rlo) * n + b0;
                acc[k] = static_cast<double>(load_if(l1, sub, in && sub < bs)) * y1 +
                         static_cast<double>(load_if(l1, sub + 16, in && sub + 16 < bs)) * y2;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                double v = acc[k];
                v += __shfl_xor(v, 8);
                v += __shfl_xor(v, 4);
                v += __shfl_xor(v, 2);
                v += __shfl_xor(v, 1);
                const int r = base + 4 * k + grp;
                if (sub == 0 && r < rhi) y[r] -= v;
            }
        }
        __syncthreads();
    }
}

// z = H_s U^{-1} L^{-1} v for one system: v, t, z in LDS (t is overwritten).
template <typename TF>
__device__ void block_precond(const BatchDesc &s, const TF *lu, const float *G, const double *cc,
                              const double *v, double *t, double *z, double *red) {
    const int n = s.n;
    for (int i = threadIdx.x; i < n; i += kBatchThreads) t[i] = v[i];
    __syncthreads();
    block_trsv<false, TF>(lu, n, t);
    block_trsv<true, TF>(lu, n, t);
    if (s.kind == RMGE_MULT_GAUSSIAN) {
        block_matvec<float>(G, n, t, z, nullptr, red);
    } else {  // z_j = sum_k c_{(j - k) mod n} t_k
        for (int j = threadIdx.x; j < n; j += kBatchThreads) {
            double acc = 0.0;
            int d = j;
            for (int k = 0; k < n; ++k) {
                acc += cc[d] * t[k];
                d = d == 0 ? n - 1 : d - 1;
            }
            z[j] = acc;
        }
        __syncthreads();
    }
}

// One system: x0 = H U^{-1} L^{-1} b, then restarted flexible GMRES on
// A d = b - A x with the right preconditioner H U^{-1} L^{-1} (basis V and
// preconditioned vectors Z in the system's Krylov workspace, classical
// Gram-Schmidt applied twice, Givens rotations by thread 0), until
// eta = ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf) <= tol or
// max_iters inner iterations.
template <typename TF>
__device__ void refine_system(const BatchDesc &s, const double *__restrict__ A,
                              const double *__restrict__ B, double *X, const TF *lu,
                              const float *G, const double *cpool, double *K,
                              const RefineParams &p, BatchOut out, double *sm) {
    const int n = s.n, tid = threadIdx.x, R = p.restart;
    double *xs = sm, *ws = sm + kBatchMaxN, *ts = sm + 2 * kBatchMaxN, *bs = sm + 3 * kBatchMaxN;
    double *cc = sm + 4 * kBatchMaxN;
    double *Hm = sm + 5 * kBatchMaxN;                       // (R + 1) x R, column j at Hm + j (R + 1)
    double *gv = Hm + (kBatchMaxRestart + 1) * kBatchMaxRestart;
    double *cs = gv + kBatchMaxRestart + 1, *sn = cs + kBatchMaxRestart;
    double *yv = sn + kBatchMaxRestart, *hv = yv + kBatchMaxRestart;  // hv: 2 x 32 dots
    double *red = hv + 2 * kBatchMaxRestart;  // [0, 8) reductions, [8], [9] scalars
    double *part = red + 16;                  // per-wave dot products, 4 x (32 + 1)
    double *V = K, *Z = K + static_cast<int64_t>(R + 1) * n;
    const double *A_s = A + s.a_off;
    const double *cpar = cpool + s.g_off;
    const float *G_s = G + s.g_off;
    for (int i = tid; i < n; i += kBatchThreads) {
        bs[i] = B[s.v_off + i];
        if (s.kind != RMGE_MULT_GAUSSIAN) cc[i] = cpar[i];
    }
    __syncthreads();
    double bmax = 0.0;
    for (int i = tid; i < n; i += kBatchThreads) bmax = fmax(bmax, fabs(bs[i]));
    const double bnorm = block_reduce(bmax, true, red);
    block_precond<TF>(s, lu, G_s, cc, bs, ts, xs, red);
    double anorm = 0.0, eta = 0.0, eta0 = -1.0;
    int used = 0;
    bool first = true, giveup = false;
    while (true) {
        // r = b - A x, eta
        block_matvec<double>(A_s, n, xs, ws, first ? &red[8] : nullptr, red);
        if (first) anorm = red[8];
        __syncthreads();
        double rinf = 0.0, xinf = 0.0, r2 = 0.0;
        for (int i = tid; i < n; i += kBatchThreads) {
            const double r = bs[i] - ws[i];
            ws[i] = r;
            rinf = fmax(rinf, fabs(r));
            xinf = fmax(xinf, fabs(xs[i]));
            r2 += r * r;
        }
        rinf = block_reduce(rinf, true, red);
        xinf = block_reduce(xinf, true, red);
        r2 = block_reduce(r2, false, red);
        const double scale = anorm * xinf + bnorm;
        eta = rinf / scale;
        if (first) {
            eta0 = eta;
            first = false;
        }
        if (!(eta > p.tol) || used >= p.max_iters || giveup || eta != eta) break;
        const double beta = sqrt(r2);
        if (!(beta > 0.0)) break;
        const double target = 0.5 * p.tol * scale;
        for (int i = tid; i < n; i += kBatchThreads) V[i] = ws[i] / beta;
        if (tid == 0) {
            for (int i = 0; i <= R; ++i) gv[i] = 0.0;
            gv[0] = beta;
        }
        __syncthreads();
        int k = 0;
        for (int j = 0; j < R && used < p.max_iters; ++j) {
            double *vj = V + static_cast<int64_t>(j) * n, *zj = Z + static_cast<int64_t>(j) * n;
            for (int i = tid; i < n; i += kBatchThreads) ts[i] = vj[i];
            __syncthreads();
            block_precond<TF>(s, lu, G_s, cc, ts, ts, ws, red);  // ws = M^{-1} v_j
            for (int i = tid; i < n; i += kBatchThreads) zj[i] = ws[i];
            __syncthreads();
            block_matvec<double>(A_s, n, ws, ts, nullptr, red);  // ts = A z_j
            // classical Gram-Schmidt, twice; the j + 1 dot products of a pass
            // eight at a time (their loads in flight together), each summed
            // over its wave, the waves' partial sums added after one barrier
            for (int pass = 0; pass < 2; ++pass) {
                for (int i0 = 0; i0 <= j; i0 += 8) {
                    double d[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) d[u] = 0.0;
                    for (int e = tid; e < n; e += kBatchThreads) {
                        const double te = ts[e];
#pragma unroll
                        for (int u = 0; u < 8; ++u)
                            if (i0 + u <= j) d[u] += V[static_cast<int64_t>(i0 + u) * n + e] * te;
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        if (i0 + u <= j) {
                            const double w = wave_sum(d[u]);
                            if ((tid & 63) == 0) part[(tid >> 6) * (kBatchMaxRestart + 1) + i0 + u] = w;
                        }
                    }
                }
                __syncthreads();
                if (tid <= j) {
                    double r = part[tid];
#pragma unroll
                    for (int w = 1; w < kBatchThreads / 64; ++w)
                        r += part[w * (kBatchMaxRestart + 1) + tid];
                    hv[pass * kBatchMaxRestart + tid] = r;
                }
                __syncthreads();
                for (int e = tid; e < n; e += kBatchThreads) {
                    double acc = ts[e];
                    for (int i = 0; i <= j; ++i)
                        acc -= hv[pass * kBatchMaxRestart + i] * V[static_cast<int64_t>(i) * n + e];
                    ts[e] = acc;
                }
                __syncthreads();
            }
            double w2 = 0.0;
            for (int e = tid; e < n; e += kBatchThreads) w2 += ts[e] * ts[e];
            const double hnext = sqrt(block_reduce(w2, false, red));
            double *vn = V + static_cast<int64_t>(j + 1) * n;
            for (int e = tid; e < n; e += kBatchThreads)
                vn[e] = hnext > 0.0 ? ts[e] / hnext : 0.0;
            if (tid == 0) {
                double *col = Hm + j * (kBatchMaxRestart + 1);
                for (int i = 0; i <= j; ++i) col[i] = hv[i] + hv[kBatchMaxRestart + i];
                col[j + 1] = hnext;
                for (int i = 0; i < j; ++i) {
                    const double a0 = col[i], b0 = col[i + 1];
                    col[i] = cs[i] * a0 + sn[i] * b0;
                    col[i + 1] = -sn[i] * a0 + cs[i] * b0;
                }
                const double a0 = col[j], b0 = col[j + 1];
                const double rr = hypot(a0, b0);
                cs[j] = rr > 0.0 ? a0 / rr : 1.0;
                sn[j] = rr > 0.0 ? b0 / rr : 0.0;
                col[j] = rr;
                col[j + 1] = 0.0;
                gv[j + 1] = -sn[j] * gv[j];
                gv[j] = cs[j] * gv[j];
                red[9] = (fabs(gv[j + 1]) <= target || !(hnext > 1e-300 * beta)) ? 1.0 : 0.0;
                if (red[9] == 0.0 && p.giveup > 0.0 && j >= 3) {
                    const double g = fabs(gv[j + 1]), q = g / beta;
                    const double more = q < 1.0 ? (j + 1) * log(target / g) / log(q) : 1e300;
                    if (used + 1 + more > p.giveup * p.max_iters) red[9] = 2.0;
                }
            }
            __syncthreads();
            ++used;
            k = j + 1;
            if (red[9] != 0.0) {
                giveup = red[9] == 2.0;
                break;
            }
        }
        if (k == 0) break;
        if (tid == 0) {  // R y = g
            for (int i = k - 1; i >= 0; --i) {
                double t = gv[i];
                for (int l = i + 1; l < k; ++l) t -= Hm[l * (kBatchMaxRestart + 1) + i] * yv[l];
                const double d = Hm[i * (kBatchMaxRestart + 1) + i];
                yv[i] = d != 0.0 ? t / d : 0.0;
            }
        }
        __syncthreads();
        for (int e = tid; e < n; e += kBatchThreads) {
            double acc = xs[e];
            for (int i = 0; i < k; ++i) acc += yv[i] * Z[static_cast<int64_t>(i) * n + e];
            xs[e] = acc;
        }
        __syncthreads();
    }
    for (int i = tid; i < n; i += kBatchThreads) X[s.v_off + i] = xs[i];
    if (tid == 0) {
        out.eta[s.sys] = eta;
        out.eta0[s.sys] = eta0;
        out.iters[s.sys] = used;
        if (!(eta <= p.tol)) out.status[s.sys] = RMGE_NOT_CONVERGED;
    }
    __syncthreads();
}

constexpr int kRefineShared =
    5 * kBatchMaxN + (kBatchMaxRestart + 1) * kBatchMaxRestart + (kBatchMaxRestart + 1) +
    5 * kBatchMaxRestart + 16 + (kBatchThreads / 64) * (kBatchMaxRestart + 1);

__global__ __launch_bounds__(kBatchThreads) void k_batch_refine(
    int count, const BatchDesc *__restrict__ d, const double *A, const double *B, double *X,
    const float *lu_pool, const float *g_pool, const double *c_pool, double *k_pool,
    RefineParams p, BatchOut out) {
    __shared__ double sm[kRefineShared];
    __shared__ int sq;
    while (true) {
        if (threadIdx.x == 0) sq = atomicAdd(out.tickets + 0, 1);
        __syncthreads();
        const int q = sq;
        __syncthreads();
        if (q >= count) return;
        const BatchDesc s = d[q];
        if (out.status[s.sys] != RMGE_OK) continue;  // broken down in the factorization
        refine_system<float>(s, A, B, X, lu_pool + s.m_off, g_pool, c_pool, k_pool + s.k_off, p,
                             out, sm);
    }
}

int bucket_of(int n) {
    return n <= 64 ? 0 : n <= 128 ? 1 : n <= 256 ? 2 : n <= 512 ? 3 : 4;
}

int log2_int(int64_t x) {
    int l = 0;
    while ((int64_t(1) << l) < x) ++l;
    return l;
}

#define BATCH_TRY(expr)                              \
    do {                                             \
        hipError_t _e = (expr);                      \
        if (_e != hipSuccess) return _e;             \
    } while (0)

template <typename T>
hipError_t upload(T **dst, const std::vector<T> &src) {
    *dst = nullptr;
    if (src.empty()) return hipSuccess;
    BATCH_TRY(hipMalloc(dst, sizeof(T) * src.size()));
    return hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
}

// ------------------------------------------------------------ FP64 fallback
//
// A system whose FP32-preconditioned refinement has not reached tol within
// max_iters inner iterations is solved again from FP64 factors (the usual
// escape of mixed-precision solvers): M = A H in FP64 with the same H (the
// Gaussian's FP32 values, or the circulant by FFT), GENP in FP64 with pivot
// blocks of 32, and the same GMRES refinement preconditioned with those
// factors.  Its result records the fallback and counts both stages'
// iterations.  The products run as whole-device launches over the marked
// systems' tiles or rows; factorization and refinement take the marked
// systems from the queue like the FP32 stage.

// Mark the systems to redo (status NOT_CONVERGED after the FP32 stage).
__global__ void k_batch_mark_fallback(int count, BatchOut out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count && out.status[i] == RMGE_NOT_CONVERGED) {
        out.status[i] = RMGE_OK;
        out.fp64[i] = 1;
    }
}

__global__ __launch_bounds__(kBatchThreads, 2) void k_batch_factor64(int count,
                                                                  const BatchDesc *__restrict__ d,
                                                                  double *m64_pool, BatchOut out) {
    __shared__ double sd[32 * 33], sinv[32];
    __shared__ int sflag, sq;
    while (true) {
        if (threadIdx.x == 0) sq = atomicAdd(out.tickets + 6, 1);
        __syncthreads();
        const int q = sq;
        __syncthreads();
        if (q >= count) return;
        const BatchDesc s = d[q];
        if (out.fp64[s.sys] == 0) continue;
        factor_system<32, double>(m64_pool + s.m_off, s.n, out.status + s.sys, out.info + s.sys,
                                  sd, sinv, &sflag);
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBatchThreads) void k_batch_refine64(
    int count, const BatchDesc *__restrict__ d, const double *A, const double *B, double *X,
    const float *g_pool, const double *c_pool, const double *m64_pool, double *k_pool,
    RefineParams p, BatchOut out) {
    __shared__ double sm[kRefineShared];
    __shared__ int sq;
    while (true) {
        if (threadIdx.x == 0) sq = atomicAdd(out.tickets + 7, 1);
        __syncthreads();
        const int q = sq;
        __syncthreads();
        if (q >= count) return;
        const BatchDesc s = d[q];
        if (out.fp64[s.sys] == 0 || out.status[s.sys] != RMGE_OK) continue;
        const int first_stage = threadIdx.x == 0 ? out.iters[s.sys] : 0;
        refine_system<double>(s, A, B, X, m64_pool + s.m_off, g_pool, c_pool, k_pool + s.k_off,
                              p, out, sm);
        if (threadIdx.x == 0) out.iters[s.sys] += first_stage;
        __syncthreads();
    }
}

}  // namespace
}  // namespace rmge

using namespace rmge;

struct rmge_batch {
    int count = 0, restart = 16, max_iters = 200;
    rmge_batch_tuning tuning{};
    std::vector<rmge_batch_system> sys;
    std::vector<BatchDesc> desc;            // queue order
    int bucket_first[RMGE_BATCH_BUCKETS] = {}, bucket_count[RMGE_BATCH_BUCKETS] = {};
                                            // queue range of each size bucket (contiguous:
                                            // the queue is in descending order of n)
    hipStream_t own = nullptr;              // stream the graph is captured on
    // draw (all systems)
    int total_chunks = 0;
    int *d_chunk_start = nullptr, *d_stream = nullptr;
    int64_t *d_cnt = nullptr, *d_poff = nullptr;
    uint64_t *d_seed = nullptr;
    // Gaussian products
    int n_gauss = 0, total_tiles = 0;
    int *d_tile_start = nullptr, *d_nsys_g = nullptr, *d_sys_g = nullptr;
    int64_t *d_aoff_g = nullptr, *d_goff_g = nullptr, *d_moff_g = nullptr;
    // circulant spectra and products
    int n_circ = 0, total_rows = 0;
    int *d_row_start = nullptr, *d_nsys_c = nullptr, *d_logl_c = nullptr, *d_sys_c = nullptr;
    int64_t *d_aoff_c = nullptr, *d_moff_c = nullptr, *d_coff_c = nullptr, *d_hoff_c = nullptr,
            *d_hhoff_c = nullptr, *d_twoff = nullptr;
    double *tw_pool = nullptr;
    // pools
    float *lu_pool = nullptr, *g_pool = nullptr;
    double *c_pool = nullptr, *h_pool = nullptr, *hh_pool = nullptr, *k_pool = nullptr;
    double *m64_pool = nullptr;  // FP64 factors of the systems that fall back
    BatchDesc *d_desc = nullptr;
    BatchOut out{};
    // captured graph and what it was captured with
    hipGraphExec_t exec = nullptr;
    const double *gA = nullptr, *gB = nullptr;
    double *gX = nullptr, gtol = 0.0;
};

namespace {

void batch_free(rmge_batch *b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    void *ptrs[] = {b->d_sys_g, b->d_sys_c,
                    b->d_chunk_start, b->d_stream, b->d_cnt, b->d_poff, b->d_seed, b->d_tile_start,
                    b->d_nsys_g, b->d_aoff_g, b->d_goff_g, b->d_moff_g, b->d_row_start,
                    b->d_nsys_c, b->d_logl_c, b->d_aoff_c, b->d_moff_c, b->d_coff_c, b->d_hoff_c,
                    b->d_hhoff_c, b->d_twoff, b->tw_pool, b->lu_pool, b->g_pool, b->c_pool,
                    b->h_pool, b->hh_pool, b->k_pool, b->m64_pool, b->out.fp64, b->d_desc,
                    b->out.status, b->out.iters,
                    b->out.eta, b->out.eta0, b->out.tickets, b->out.info};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (b->own) (void)hipStreamDestroy(b->own);
    delete b;
}

rmge_status batch_status(hipError_t e) {
    if (e == hipSuccess) return RMGE_OK;
    return e == hipErrorOutOfMemory ? RMGE_ENOMEM : RMGE_EDEVICE;
}

// Panel widths from the tuning, into the queue descriptors (host and device).
hipError_t apply_tuning(rmge_batch *b) {
    for (BatchDesc &d : b->desc) d.nb = b->tuning.nb[bucket_of(d.n)];
    return hipMemcpy(b->d_desc, b->desc.data(), sizeof(BatchDesc) * b->desc.size(),
                     hipMemcpyHostToDevice);
}

bool valid_nb(int nb) { return nb == 16 || nb == 32 || nb == 64; }

// The chain up to the products (every multiplier drawn and applied).
hipError_t enqueue_products(rmge_batch *b, const double *A, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_reset, dim3(static_cast<unsigned>((b->count + 255) / 256)),
                       dim3(256), 0, s, b->count, b->out);
    BATCH_TRY(hipGetLastError());
    BATCH_TRY(batch_normals(b->count, b->total_chunks, b->d_chunk_start, b->d_cnt, b->d_stream,
                            b->d_seed, b->d_poff, b->g_pool, b->c_pool, s));
    BATCH_TRY(batch_fft_spectra(b->n_circ, b->d_nsys_c, b->d_logl_c, b->d_coff_c, b->d_hoff_c,
                                b->d_hhoff_c, b->d_twoff, b->c_pool, b->h_pool, b->hh_pool,
                                b->tw_pool, s));
    BATCH_TRY(batch_gemm_f32(b->n_gauss, b->total_tiles, b->d_tile_start, b->d_nsys_g,
                             b->d_aoff_g, b->d_goff_g, b->d_moff_g, A, b->g_pool, b->lu_pool, s));
    return batch_fft_rows<float>(b->n_circ, b->total_rows, b->d_row_start, b->d_nsys_c, nullptr,
                                 nullptr, b->d_logl_c, b->d_aoff_c, b->d_moff_c, b->d_hhoff_c,
                                 b->d_twoff, A, b->hh_pool, b->tw_pool, b->lu_pool, s);
}

int grid_for(int count, int per_cu) {
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const int g = per_cu * ncu;
    return count < g ? count : g;
}

// Factor size bucket bk (a contiguous range of the queue) with its panel width.
hipError_t enqueue_factor_bucket(rmge_batch *b, int bk, hipStream_t s) {
    const int first = b->bucket_first[bk], cnt = b->bucket_count[bk];
    if (cnt <= 0) return hipSuccess;
    const dim3 grid(static_cast<unsigned>(grid_for(cnt, 4))), block(kBatchThreads);
    int *ticket = b->out.tickets + 1 + bk;
    switch (b->tuning.nb[bk]) {
    case 16:
        hipLaunchKernelGGL(k_batch_factor<16>, grid, block, 0, s, cnt, b->d_desc + first,
                           b->lu_pool, b->out, ticket);
        break;
    case 32:
        hipLaunchKernelGGL(k_batch_factor<32>, grid, block, 0, s, cnt, b->d_desc + first,
                           b->lu_pool, b->out, ticket);
        break;
    default:
        hipLaunchKernelGGL(k_batch_factor<64>, grid, block, 0, s, cnt, b->d_desc + first,
                           b->lu_pool, b->out, ticket);
        break;
    }
    return hipGetLastError();
}

hipError_t enqueue_refine(rmge_batch *b, const double *A, const double *B, double *X, double tol,
                          hipStream_t s) {
    // the FP64 stage follows, so a system projected to need more than 1.5
    // times the budget is handed to it early (4096-system batch, budget 16:
    // 187.3 -> 177.4 ms a step, 973 -> 1032 systems to the FP64 stage)
    RefineParams p{b->restart, b->max_iters, tol, 1.5};
    hipLaunchKernelGGL(k_batch_refine, dim3(static_cast<unsigned>(grid_for(b->count, 3))),
                       dim3(kBatchThreads), 0, s, b->count, b->d_desc, A, B, X, b->lu_pool,
                       b->g_pool, b->c_pool, b->k_pool, p, b->out);
    return hipGetLastError();
}

hipError_t enqueue_fallback(rmge_batch *b, const double *A, const double *B, double *X,
                            double tol, hipStream_t s) {
    RefineParams p{b->restart, b->max_iters, tol, 0.0};
    hipLaunchKernelGGL(k_batch_mark_fallback, dim3(static_cast<unsigned>((b->count + 255) / 256)),
                       dim3(256), 0, s, b->count, b->out);
    BATCH_TRY(hipGetLastError());
    BATCH_TRY(batch_gemm_f64(b->n_gauss, b->total_tiles, b->d_tile_start, b->d_nsys_g, b->d_sys_g,
                             b->out.fp64, b->d_aoff_g, b->d_goff_g, b->d_moff_g, A, b->g_pool,
                             b->m64_pool, s));
    BATCH_TRY(batch_fft_rows<double>(b->n_circ, b->total_rows, b->d_row_start, b->d_nsys_c,
                                     b->d_sys_c, b->out.fp64, b->d_logl_c, b->d_aoff_c,
                                     b->d_moff_c, b->d_hhoff_c, b->d_twoff, A, b->hh_pool,
                                     b->tw_pool, b->m64_pool, s));
    hipLaunchKernelGGL(k_batch_factor64, dim3(static_cast<unsigned>(grid_for(b->count, 4))),
                       dim3(kBatchThreads), 0, s, b->count, b->d_desc, b->m64_pool, b->out);
    BATCH_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_batch_refine64, dim3(static_cast<unsigned>(grid_for(b->count, 3))),
                       dim3(kBatchThreads), 0, s, b->count, b->d_desc, A, B, X, b->g_pool,
                       b->c_pool, b->m64_pool, b->k_pool, p, b->out);
    return hipGetLastError();
}

hipError_t enqueue_all(rmge_batch *b, const double *A, const double *B, double *X, double tol,
                       hipStream_t s) {
    BATCH_TRY(enqueue_products(b, A, s));
    for (int bk = RMGE_BATCH_BUCKETS - 1; bk >= 0; --bk) BATCH_TRY(enqueue_factor_bucket(b, bk, s));
    BATCH_TRY(enqueue_refine(b, A, B, X, tol, s));
    return enqueue_fallback(b, A, B, X, tol, s);
}

bool device_is_gfx950() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, dev) != hipSuccess) return false;
    return std::strncmp(pr.gcnArchName, "gfx950", 6) == 0;
}

rmge_status batch_build(rmge_batch *b) {
    const int count = b->count;
    // queue: descending order, then the caller's order
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return b->sys[x].n > b->sys[y].n; });
    int64_t lu_total = 0, g_total = 0, c_total = 0, h_total = 0, hh_total = 0, k_total = 0;
    std::vector<int> chunk_start{0}, stream_of, tile_start{0}, nsys_g, sys_g, row_start{0}, nsys_c,
        sys_c, logl_c;
    std::vector<int64_t> cnt, poff, aoff_g, goff_g, moff_g, aoff_c, moff_c, coff_c, hoff_c, hhoff_c;
    std::vector<uint64_t> seed;
    for (int q = 0; q < count; ++q) {
        const rmge_batch_system &y = b->sys[order[q]];
        const int64_t n = y.n;
        BatchDesc d{};
        d.n = y.n;
        d.kind = y.kind;
        d.sys = order[q];
        d.a_off = y.a_off;
        d.v_off = y.v_off;
        d.m_off = lu_total;
        lu_total += n * n;
        d.k_off = k_total;
        k_total += static_cast<int64_t>(2 * b->restart + 1) * n;
        const int bk = bucket_of(y.n);
        if (b->bucket_count[bk]++ == 0) b->bucket_first[bk] = q;
        if (y.kind == RMGE_MULT_GAUSSIAN) {
            d.g_off = g_total;
            g_total += n * n;
            cnt.push_back(n * n);
            stream_of.push_back(1);
            const int64_t tiles = ((n + 63) / 64) * ((n + 63) / 64);
            tile_start.push_back(tile_start.back() + static_cast<int>(tiles));
            nsys_g.push_back(y.n);
            sys_g.push_back(order[q]);
            aoff_g.push_back(y.a_off);
            goff_g.push_back(d.g_off);
            moff_g.push_back(d.m_off);
        } else {
            d.g_off = c_total;
            c_total += n;
            cnt.push_back(n);
            stream_of.push_back(2);
            const int64_t m = (n >= 2 && (n & (n - 1)) == 0) ? n : std::max<int64_t>(2, int64_t(1) << log2_int(2 * n - 1));
            nsys_c.push_back(y.n);
            sys_c.push_back(order[q]);
            logl_c.push_back(log2_int(m / 2));
            aoff_c.push_back(y.a_off);
            moff_c.push_back(d.m_off);
            coff_c.push_back(d.g_off);
            hoff_c.push_back(h_total);
            h_total += m;
            hhoff_c.push_back(hh_total);
            hh_total += m / 2 + 1;
            row_start.push_back(row_start.back() + y.n);
        }
        poff.push_back(d.g_off);
        seed.push_back(y.seed);
        chunk_start.push_back(chunk_start.back() + static_cast<int>((cnt.back() + 1023) / 1024));
        b->desc.push_back(d);
    }
    b->total_chunks = chunk_start.back();
    b->n_gauss = static_cast<int>(nsys_g.size());
    b->total_tiles = tile_start.back();
    b->n_circ = static_cast<int>(nsys_c.size());
    b->total_rows = row_start.back();
    // twiddle tables, one per period present (log2 L = 0 .. 10)
    std::vector<int64_t> twoff(11, 0);
    int64_t tw_total = 0;
    for (int l = 0; l <= 10; ++l) {
        twoff[l] = tw_total;
        tw_total += (int64_t(1) << l) + 1;
    }
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) {
        if (e == hipSuccess) e = x;
    };
    chk(hipMalloc(&b->tw_pool, sizeof(double) * 2 * tw_total));
    for (int l = 0; l <= 10 && e == hipSuccess; ++l)
        chk(fft_twiddles(2 << l, b->tw_pool + 2 * twoff[l], nullptr));
    chk(upload(&b->d_chunk_start, chunk_start));
    chk(upload(&b->d_stream, stream_of));
    chk(upload(&b->d_cnt, cnt));
    chk(upload(&b->d_poff, poff));
    chk(upload(&b->d_seed, seed));
    chk(upload(&b->d_tile_start, tile_start));
    chk(upload(&b->d_nsys_g, nsys_g));
    chk(upload(&b->d_sys_g, sys_g));
    chk(upload(&b->d_aoff_g, aoff_g));
    chk(upload(&b->d_goff_g, goff_g));
    chk(upload(&b->d_moff_g, moff_g));
    chk(upload(&b->d_row_start, row_start));
    chk(upload(&b->d_sys_c, sys_c));
    chk(upload(&b->d_nsys_c, nsys_c));
    chk(upload(&b->d_logl_c, logl_c));
    chk(upload(&b->d_aoff_c, aoff_c));
    chk(upload(&b->d_moff_c, moff_c));
    chk(upload(&b->d_coff_c, coff_c));
    chk(upload(&b->d_hoff_c, hoff_c));
    chk(upload(&b->d_hhoff_c, hhoff_c));
    chk(upload(&b->d_twoff, twoff));
    chk(hipMalloc(&b->lu_pool, sizeof(float) * std::max<int64_t>(1, lu_total)));
    chk(hipMalloc(&b->m64_pool, sizeof(double) * std::max<int64_t>(1, lu_total)));
    chk(hipMalloc(&b->g_pool, sizeof(float) * std::max<int64_t>(1, g_total)));
    chk(hipMalloc(&b->c_pool, sizeof(double) * std::max<int64_t>(1, c_total)));
    chk(hipMalloc(&b->h_pool, sizeof(double) * std::max<int64_t>(1, h_total)));
    chk(hipMalloc(&b->hh_pool, sizeof(double) * 2 * std::max<int64_t>(1, hh_total)));
    chk(hipMalloc(&b->k_pool, sizeof(double) * std::max<int64_t>(1, k_total)));
    chk(hipMalloc(&b->d_desc, sizeof(BatchDesc) * count));
    chk(hipMalloc(&b->out.status, sizeof(int) * count));
    chk(hipMalloc(&b->out.iters, sizeof(int) * count));
    chk(hipMalloc(&b->out.eta, sizeof(double) * count));
    chk(hipMalloc(&b->out.eta0, sizeof(double) * count));
    chk(hipMalloc(&b->out.tickets, sizeof(int) * 8));
    chk(hipMalloc(&b->out.info, sizeof(int64_t) * count));
    chk(hipMalloc(&b->out.fp64, sizeof(int) * count));
    if (e == hipSuccess) e = apply_tuning(b);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking);
    return batch_status(e);
}

}  // namespace

extern "C" {

rmge_status rmge_batch_create(const rmge_batch_system *systems, int32_t count,
                              const rmge_batch_tuning *tuning, int32_t restart, int32_t max_iters,
                              rmge_batch **out) {
    if (!systems || !out || count < 1 || restart < 1 || restart > kBatchMaxRestart ||
        max_iters < 0)
        return RMGE_EINVAL;
    for (int i = 0; i < count; ++i) {
        const rmge_batch_system &y = systems[i];
        if (y.n < 1 || y.n > kBatchMaxN || y.a_off < 0 || y.v_off < 0 ||
            (y.kind != RMGE_MULT_GAUSSIAN && y.kind != RMGE_MULT_CIRCULANT))
            return RMGE_EINVAL;
    }
    if (tuning)
        for (int bk = 0; bk < RMGE_BATCH_BUCKETS; ++bk)
            if (!valid_nb(tuning->nb[bk])) return RMGE_EINVAL;
    if (!device_is_gfx950()) return RMGE_EDEVICE;
    rmge_batch *b = new (std::nothrow) rmge_batch();
    if (!b) return RMGE_ENOMEM;
    b->count = count;
    b->restart = restart;
    b->max_iters = max_iters;
    b->sys.assign(systems, systems + count);
    const rmge_batch_tuning dflt{{32, 32, 32, 64, 64}};
    b->tuning = tuning ? *tuning : dflt;
    const rmge_status rs = batch_build(b);
    if (rs != RMGE_OK) {
        batch_free(b);
        return rs;
    }
    *out = b;
    return RMGE_OK;
}

rmge_status rmge_batch_run(rmge_batch *b, const double *A, const double *B, double *X, double tol,
                           void *hip_stream) {
    if (!b || !A || !B || !X || !(tol > 0.0)) return RMGE_EINVAL;
    return batch_status(enqueue_all(b, A, B, X, tol, static_cast<hipStream_t>(hip_stream)));
}

rmge_status rmge_batch_run_timed(rmge_batch *b, const double *A, const double *B, double *X,
                                 double tol, void *hip_stream, double *ms4) {
    if (!b || !A || !B || !X || !(tol > 0.0) || !ms4) return RMGE_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    hipError_t e = hipSuccess;
    for (hipEvent_t &x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    if (e == hipSuccess) e = hipEventRecord(ev[0], s);
    if (e == hipSuccess) e = enqueue_products(b, A, s);
    if (e == hipSuccess) e = hipEventRecord(ev[1], s);
    for (int bk = RMGE_BATCH_BUCKETS - 1; bk >= 0 && e == hipSuccess; --bk)
        e = enqueue_factor_bucket(b, bk, s);
    if (e == hipSuccess) e = hipEventRecord(ev[2], s);
    if (e == hipSuccess) e = enqueue_refine(b, A, B, X, tol, s);
    if (e == hipSuccess) e = hipEventRecord(ev[3], s);
    if (e == hipSuccess) e = enqueue_fallback(b, A, B, X, tol, s);
    if (e == hipSuccess) e = hipEventRecord(ev[4], s);
    if (e == hipSuccess) e = hipEventSynchronize(ev[4]);
    for (int i = 0; i < 4 && e == hipSuccess; ++i) {
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
        ms4[i] = ms;
    }
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    return batch_status(e);
}

rmge_status rmge_batch_graph_run(rmge_batch *b, const double *A, const double *B, double *X,
                                 double tol, void *hip_stream) {
    if (!b || !A || !B || !X || !(tol > 0.0)) return RMGE_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (!b->exec || b->gA != A || b->gB != B || b->gX != X || b->gtol != tol) {
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return batch_status(e);
        const hipError_t e1 = enqueue_all(b, A, B, X, tol, b->own);
        e = hipStreamEndCapture(b->own, &g);
        if (e1 != hipSuccess || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return batch_status(e1 != hipSuccess ? e1 : e);
        }
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            b->exec = nullptr;
            return batch_status(e);
        }
        b->gA = A;
        b->gB = B;
        b->gX = X;
        b->gtol = tol;
    }
    return batch_status(hipGraphLaunch(b->exec, s));
}

rmge_status rmge_batch_results(const rmge_batch *b, int32_t *status, double *eta, double *eta0,
                               int32_t *iters, int64_t *info, int32_t *fp64, void *hip_stream) {
    if (!b) return RMGE_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipStreamSynchronize(s);
    const size_t c = static_cast<size_t>(b->count);
    if (e == hipSuccess && status) e = hipMemcpy(status, b->out.status, 4 * c, hipMemcpyDeviceToHost);
    if (e == hipSuccess && eta) e = hipMemcpy(eta, b->out.eta, 8 * c, hipMemcpyDeviceToHost);
    if (e == hipSuccess && eta0) e = hipMemcpy(eta0, b->out.eta0, 8 * c, hipMemcpyDeviceToHost);
    if (e == hipSuccess && iters) e = hipMemcpy(iters, b->out.iters, 4 * c, hipMemcpyDeviceToHost);
    if (e == hipSuccess && info) e = hipMemcpy(info, b->out.info, 8 * c, hipMemcpyDeviceToHost);
    if (e == hipSuccess && fp64) e = hipMemcpy(fp64, b->out.fp64, 4 * c, hipMemcpyDeviceToHost);
    return batch_status(e);
}

rmge_status rmge_batch_get_tuning(const rmge_batch *b, rmge_batch_tuning *t) {
    if (!b || !t) return RMGE_EINVAL;
    *t = b->tuning;
    return RMGE_OK;
}

rmge_status rmge_batch_set_tuning(rmge_batch *b, const rmge_batch_tuning *t) {
    if (!b || !t) return RMGE_EINVAL;
    for (int bk = 0; bk < RMGE_BATCH_BUCKETS; ++bk)
        if (!valid_nb(t->nb[bk])) return RMGE_EINVAL;
    b->tuning = *t;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);  // the graph bakes the descriptors' launch
    b->exec = nullptr;
    return batch_status(apply_tuning(b));
}

rmge_status rmge_batch_autotune(rmge_batch *b, const double *A, void *hip_stream,
                                rmge_batch_tuning *best, double *ms_bucket) {
    if (!b || !A || !best) return RMGE_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int cand[3] = {16, 32, 64};
    rmge_batch_tuning keep = b->tuning, result = b->tuning;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    for (int bk = 0; bk < RMGE_BATCH_BUCKETS && e == hipSuccess; ++bk) {
        const int cnt = b->bucket_count[bk];
        double best_ms = -1.0;
        for (int c = 0; c < 3 && e == hipSuccess && cnt > 0; ++c) {
            rmge_batch_tuning t = keep;
            t.nb[bk] = cand[c];
            b->tuning = t;
            e = apply_tuning(b);
            float ms = 0.0f;
            for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // the first run warms up
                e = enqueue_products(b, A, s);  // the factorization overwrites the products
                if (e == hipSuccess) e = hipEventRecord(e0, s);
                if (e == hipSuccess) e = enqueue_factor_bucket(b, bk, s);
                if (e == hipSuccess) e = hipEventRecord(e1, s);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            }
            if (e == hipSuccess && (best_ms < 0.0 || ms < best_ms)) {
                best_ms = ms;
                result.nb[bk] = cand[c];
            }
        }
        if (ms_bucket) ms_bucket[bk] = best_ms;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    b->tuning = result;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
    if (e == hipSuccess) e = apply_tuning(b);
    *best = result;
    return batch_status(e);
}

rmge_status rmge_batch_factors_lu(const rmge_batch *b, int32_t index, double *LU, int64_t ld,
                                  void *hip_stream) {
    if (!b || !LU || index < 0 || index >= b->count) return RMGE_EINVAL;
    const int n = b->sys[index].n;
    if (ld < n) return RMGE_EINVAL;
    int64_t m_off = -1;
    for (const BatchDesc &d : b->desc)
        if (d.sys == index) m_off = d.m_off;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipError_t e = convert_2d<float, double>(b->lu_pool + m_off, n, LU, ld, n, n, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return batch_status(e);
}

void rmge_batch_destroy(rmge_batch *b) { batch_free(b); }

}  // extern "C"
