// C ABI of the library: handle management and the order of the method's steps.
//
//   factor:  H from the seed  ->  M = A H  ->  block elimination with no
//            pivoting on M (eq. eqgenp with pivot blocks of `block` columns),
//            or with partial pivoting confined to the small diagonal blocks
//            where the recursion stops (Section 3, after eq. eqgenpin);
//   solve:   x = H U^{-1} L^{-1} b (Fact faprepr), then refinement
//            r = b - A x (FP64), x += H U^{-1} L^{-1} r (Section 8.1);
//   adjoint: y = L^{-T} U^{-T} H^T w.
//
// Device memory layout (one handle, factor precision T):
//   lu    n x ld  (ld = n rounded up to 64)  the packed factors, over M
//   mult  GAUSSIAN: n x n of T, G row-major; CIRCULANT/TOEPLITZ: parameters,
//         the period-m kernel h, its half spectrum and the twiddle table
//   inv   two buffers (the look-ahead panel and the current one), each the
//         inverses of the 32 x 32 diagonal sub-blocks of a pivot block's L and
//         U, compact (256 x 32 each)
//   sinv  the same for every aligned 32-row diagonal sub-block of the final
//         L and U (2 x round_up(n, 256) x 32), used by the solves with several
//         right-hand sides and the adjoint solves
//   binv  FP64 inverses of the 128 x 128 diagonal blocks of L and U, and
//         their products with the adjacent coupling blocks
//         (4 x round_up(n, 128) x 128), used by the single right-hand-side
//         solves
//   piv   n ints (pivoted variant): row t of the factors is row piv[t] of M
//   solve workspace, grown on demand: two n x nrhs of T, one n x nrhs FP64
//         residual, norms
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/rmge.h"
#include "rmge_impl.h"

using namespace rmge;

struct rmge_factors {
    int64_t n = 0, lda = 0, ld = 0;
    int32_t kind = 0, prec = 0, block = 0, pivot = 0;
    uint64_t seed = 0;
    hipStream_t stream = nullptr;
    const double *A = nullptr;
    void *lu = nullptr;
    void *G = nullptr;         // GAUSSIAN multiplier (T)
    float *a32 = nullptr;      // FP32 GAUSSIAN: A rounded to FP32 (n x ld) for the product
    bool split16 = false;       // RMGE_F32_BF16X2 with a GAUSSIAN multiplier
    uint16_t *a16 = nullptr;    // split16: A_h then A_l, BF16 bits, rows16 x ldk16 each
    uint16_t *ht16 = nullptr;   // split16: H^T as BF16 bits, rows16 x ldk16
    int64_t rows16 = 0, ldk16 = 0;
    // BF16 Schur updates (RMGE_F32_BF16X2: three-term split at FP32 accuracy,
    // trailing blocks of kSplitUpdateMin rows and more; RMGE_BF16: operands
    // rounded once to BF16, every bulk update): upd_terms = 3 or 1, 0 if none
    int upd_terms = 0;
    uint16_t *u16 = nullptr;    // the BF16 terms of the update's operands
    int64_t urows = 0, uldk = 0;  // (2 * upd_terms slabs of urows x uldk)
    double *wht = nullptr;      // split16: partial sums of H y over Ht
    double *params = nullptr;  // structured multiplier parameters
    double *hker = nullptr;    // period-m kernel
    double *hhat = nullptr;    // half spectrum (m/2 + 1 complex)
    double *tw = nullptr;      // twiddles (m/2 + 1 complex)
    int m = 0;
    void *inv = nullptr;
    void *sinv = nullptr;  // solve inverses: L part, then U part (sinv_rows rows each)
    int64_t sinv_rows = 0;
    double *binv = nullptr;  // block inverses: L part, then U part (binv_rows rows each)
    int64_t binv_rows = 0;
    bool binv_done = false;  // formed by the first one-RHS solve after a factorization
    int *piv = nullptr;  // pivoted variant: P M = L U with row t = row piv[t] of M
    DevStatus *st = nullptr;
    double *scal = nullptr;  // [0] max|U| [1] min|u_kk| [2] max|M| [3] ||A||_inf [4] ||A||_1
    // solve workspace
    int64_t ws_nrhs = 0;
    double *wy = nullptr, *wx = nullptr;  // solve vectors (FP64 for every factor type)
    double *wr = nullptr, *wnorm = nullptr;
    double *wt = nullptr;
    int64_t wt_size = 0;
    int *wsync = nullptr;  // persistent solves: ticket counter, error word
    // Krylov workspace (FP64): basis V (restart + 1 vectors), preconditioned
    // vectors Z (restart), residual, partial sums and small device vectors
    double *kv = nullptr;
    int kv_restart = 0;
    double *kb = nullptr;  // block Krylov workspace (several right-hand sides)
    int64_t kb_words = 0;
    // host copies
    DevStatus host_st{-1, 0, 0};
    bool stats_done = false;
    bool anorm_done = false, anorm1_done = false;
    double anorm = 0.0, anorm1 = 0.0;  // ||A||_inf, ||A||_1 (= ||A^T||_inf)
    rmge_factor_stats stats{};
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    hipStream_t side = nullptr;  // look-ahead stream (default priority)
    hipStream_t main = nullptr;  // set when the side stream owns reserved CUs
    hipStream_t aux = nullptr;   // the reserved CUs' share of a Schur update
    int cus_main = 0, cus_side = 0;
    double aux_scale = 0.0;  // safety factor on the reserved CUs' share (0: none)
    hipEvent_t ev_narrow = nullptr, ev_panel = nullptr, ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t ev_aux = nullptr;
    // the bulk Schur updates' device time: an event pair around each launch
    // (created when the factorization has at most kUpdEvents steps)
    std::vector<hipEvent_t> upd_ev;
    double upd_flops = 0.0, ms_update = 0.0;
};

namespace {

constexpr int kSub = 32;      // rows of the inverted diagonal sub-blocks
constexpr int kUpdEvents = 512;  // steps of a factorization whose updates are timed
// Compute units reserved for the look-ahead stream.  A queue masked to 248 of
// the 256 units dispatches one-round grids as if it had 224 (the mask is
// evened out over the 32 shader arrays), so reserving 32 costs the main
// stream no more than reserving 8.
constexpr int kSideCUs = 32;
// Split-BF16 handles: trailing blocks of at least this many rows take the
// three-term BF16 Schur update (smaller ones fill too few 256 x 256 tiles to
// beat the FP32 kernels)
constexpr int64_t kSplitUpdateMin = 2048;

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

rmge_status from_hip(hipError_t e) {
    if (e == hipSuccess) return RMGE_OK;
    if (e == hipErrorOutOfMemory) return RMGE_ENOMEM;
    return RMGE_EDEVICE;
}

#define RMGE_TRY(expr)                                         \
    do {                                                       \
        hipError_t _e = (expr);                                \
        if (_e != hipSuccess) {                                \
            if (std::getenv("RMGE_DEBUG"))                     \
                std::fprintf(stderr, "rmge: %s failed: %s\n", #expr, hipGetErrorString(_e)); \
            return from_hip(_e);                               \
        }                                                      \
    } while (0)

#define HIP_TRY(expr)                      \
    do {                                   \
        hipError_t _e = (expr);            \
        if (_e != hipSuccess) return _e;   \
    } while (0)

size_t elem_size(int prec) { return prec == RMGE_F32 ? sizeof(float) : sizeof(double); }

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

int64_t next_pow2(int64_t x) {
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Multipliers applied by FFT: circulants (Gaussian or unitary first column) and Toeplitz.
bool is_fft_kind(int kind) {
    return kind == RMGE_MULT_CIRCULANT || kind == RMGE_MULT_TOEPLITZ ||
           kind == RMGE_MULT_UNITARY_CIRCULANT;
}

bool is_circulant(int kind) {
    return kind == RMGE_MULT_CIRCULANT || kind == RMGE_MULT_UNITARY_CIRCULANT;
}

// FFT period for the structured multipliers (0 if unsupported).
int fft_period(int kind, int64_t n) {
    int64_t m;
    if (is_circulant(kind) && n >= 2 && is_pow2(n))
        m = n;
    else
        m = next_pow2(2 * n - 1);
    if (m < 2) m = 2;
    return m <= 16384 ? static_cast<int>(m) : 0;
}

bool device_ok() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return false;
    return std::strncmp(p.gcnArchName, "gfx950", 6) == 0;
}

__global__ void k_reset(DevStatus *st, double *scal) {
    st->info = -1;
    st->code = 0;
    st->pad = 0;
    scal[0] = 0.0;
    scal[1] = INFINITY;
    scal[2] = 0.0;
}

template <typename T>
struct Prec;
template <>
struct Prec<double> {
    static hipError_t gemm(int shape, int64_t M, int64_t N, int64_t K, double alpha,
                           const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
                           double *C, int64_t ldc, const int *abort, hipStream_t s) {
        return gemm_f64(shape, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, abort, s);
    }
    static hipError_t gemm_a64(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda,
                               const double *B, int64_t ldb, double *C, int64_t ldc,
                               double *absmax, hipStream_t s) {
        return gemm_f64(kGemmProduct, M, N, K, 1.0, A, lda, B, ldb, 0.0, C, ldc, nullptr, s,
                        absmax);
    }
    static hipError_t normals(double *out, int64_t count, uint64_t seed, uint64_t stream,
                              hipStream_t s) {
        return launch_normals_f64(out, count, seed, stream, s);
    }
};
template <>
struct Prec<float> {
    static hipError_t gemm(int shape, int64_t M, int64_t N, int64_t K, float alpha, const float *A,
                           int64_t lda, const float *B, int64_t ldb, float beta, float *C,
                           int64_t ldc, const int *abort, hipStream_t s) {
        return gemm_f32(shape, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, abort, s);
    }
    static hipError_t gemm_a64(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda,
                               const float *B, int64_t ldb, float *C, int64_t ldc, double *absmax,
                               hipStream_t s) {
        return gemm_f32_a64(kGemmProduct, M, N, K, 1.0f, A, lda, B, ldb, 0.0f, C, ldc, nullptr, s,
                            absmax);
    }
    static hipError_t normals(float *out, int64_t count, uint64_t seed, uint64_t stream,
                              hipStream_t s) {
        return launch_normals_f32(out, count, seed, stream, s);
    }
};

// ------------------------------------------------------------------ factor

// Factor the b x b pivot block at `a` in place and leave the inverses of the
// 32 x 32 diagonal sub-blocks of its factors in Linv, Uinv (compact, 32 columns).
// Blocks wider than the LDS leaf are split once: B = [[Ba, Bab], [Bba, Bb]] is
// eliminated as in eq. eqgenp with pivot block Ba.
template <typename T>
hipError_t factor_pivot_block(rmge_factors *f, T *a, int b, int64_t k0, T *Linv, T *Uinv,
                              hipStream_t s) {
    const int64_t ld = f->ld;
    const int *abort = &f->st->code;
    int *piv = f->pivot ? f->piv : nullptr;
    if (b <= kLeaf) return leaf_lu<T>(a, ld, b, Linv, Uinv, k0, f->st, piv, s);
    const int b1 = kLeaf, b2 = b - kLeaf;
    HIP_TRY(leaf_lu<T>(a, ld, b1, Linv, Uinv, k0, f->st, piv, s));
    // Bab <- La^{-1} Pa Bab ; Bba <- Bba Ua^{-1} (one launch) ; Bb <- Bb - Bba Bab
    HIP_TRY(trsm_pair<T>(a, ld, b1, a + b1, ld, b2, Linv, piv ? piv + k0 : nullptr, k0,
                         a + b1 * ld, ld, b2, Uinv, abort, s));
    HIP_TRY(Prec<T>::gemm(kGemmUpdate, b2, b2, b1, T(-1), a + b1 * ld, ld, a + b1, ld, T(1),
                          a + b1 * ld + b1, ld, abort, s));
    HIP_TRY(leaf_lu<T>(a + b1 * ld + b1, ld, b2, Linv + b1 * kSub, Uinv + b1 * kSub, k0 + b1,
                       f->st, piv, s));
    // the second block's exchanges reach Bba now: the solves with this pivot
    // block's L (block row, next step) need its rows in pivot order
    if (piv) {
        T *base = static_cast<T *>(f->lu);
        HIP_TRY(permute_rows<T>(base, ld, k0 + b1, b2, k0, k0 + b1, piv, abort, s));
    }
    return hipSuccess;
}

// Columns of a wide Schur update (r rows, w columns, depth b) handed to the
// reserved compute units.  They are free once the side stream has factored the
// next pivot block, about t_side after the narrow update; with Cm main and Cs
// reserved units the two parts end together when the reserved share is
// Cs / (Cm + Cs) * (1 - t_side / T), T the update's time on the main units
// alone.  Rates and t_side are nominal (measured on the update kernels and
// the pivot-block chain at block 256); aux_scale scales the share (1 measured
// best against 0.9 and 1.1; the main stream waits for the reserved part, so a
// share too large costs more than one too small).  The two parts share L2 and
// HBM bandwidth, so the main part slows a little while both run.
template <typename T>
int64_t aux_columns(const rmge_factors *f, int64_t r, int64_t w, int b) {
    if (f->aux == nullptr || f->aux_scale <= 0.0 || f->cus_side <= 0 || f->cus_main <= 0) return 0;
    const double per_cu = sizeof(T) == 8 ? 2.3e11 : 4.4e11;  // update flop/s per compute unit
    const double t_side = (sizeof(T) == 8 ? 220e-6 : 160e-6) * b / 256.0;
    const double t_full = 2.0 * static_cast<double>(r) * static_cast<double>(w) * b /
                          (per_cu * f->cus_main);
    if (t_full <= t_side) return 0;
    const double share = f->aux_scale * f->cus_side / static_cast<double>(f->cus_main + f->cus_side) *
                         (1.0 - t_side / t_full);
    const int64_t wa = static_cast<int64_t>(share * static_cast<double>(w)) / 128 * 128;
    return wa < 128 ? 0 : (wa > w ? w : wa);
}

// Right-looking block elimination with no pivoting (eq. eqgenp applied to
// pivot blocks of f->block columns) with one panel of look-ahead.  Step k:
//   main stream:  (once the side stream has factored pivot block k)
//                 D <- D U_B^{-1} for the column below it;
//                 C <- L_B^{-1} C for the block row right of it;
//                 Schur update of the next panel's columns only;
//   side stream:  (after that narrow update) factor the next pivot block;
//   main stream:  Schur update E <- E - D C of all remaining columns, which
//                 runs while the side stream works on the next pivot block.
// The side stream's kernels are one or a few workgroups each; it owns a few
// reserved compute units (CU masks, same priority), because a wide update
// keeps every register file of the others full and would starve it.
// The update E - (D U_B^{-1})(L_B^{-1} C) is E - D B^{-1} C of eq. eqgenp.
// Once the next pivot block is factored the reserved units are idle, so an
// aux stream on them takes the last columns of the wide update (aux_columns);
// the main stream waits for that part before the next step.
// Pivoted variant: P_B B = L_B U_B inside the pivot block, the block row is
// read through P_B (L_B^{-1} P_B C), the rows below are untouched, and one
// pass at the end applies the exchanges to the multipliers left of each block.
// Inverses of the pivot blocks' diagonal sub-blocks alternate between two
// buffers so the side stream never overwrites those the main stream reads.
template <typename T>
hipError_t genp_blocked(rmge_factors *f) {
    T *a = static_cast<T *>(f->lu);
    const int64_t n = f->n, ld = f->ld;
    const int nb = f->block;
    T *inv = static_cast<T *>(f->inv);
    const int64_t invsz = 2 * kMaxBlock * kSub;
    const int *abort = &f->st->code;
    hipStream_t s0 = f->main ? f->main : f->stream, s1 = f->side;
    if (f->main) {
        HIP_TRY(hipEventRecord(f->ev_fork, f->stream));
        HIP_TRY(hipStreamWaitEvent(s0, f->ev_fork, 0));
    }
    auto Linv = [&](int64_t step) { return inv + (step & 1) * invsz; };
    auto Uinv = [&](int64_t step) { return inv + (step & 1) * invsz + kMaxBlock * kSub; };

    // pivot block 0 on the main stream
    HIP_TRY(factor_pivot_block<T>(f, a, static_cast<int>(n < nb ? n : nb), 0, Linv(0), Uinv(0),
                                  s0));
    int64_t step = 0;
    bool aux_pending = false;  // the reserved units' part of the last wide update
    for (int64_t k = 0; k < n; k += nb, ++step) {
        const int b = static_cast<int>((n - k) < nb ? (n - k) : nb);
        if (k > 0) HIP_TRY(hipStreamWaitEvent(s0, f->ev_panel, 0));
        if (aux_pending) {
            HIP_TRY(hipStreamWaitEvent(s0, f->ev_aux, 0));
            aux_pending = false;
        }
        if (k + b >= n) break;
        const int64_t r = n - k - b;
        const int bn = static_cast<int>(r < nb ? r : nb);  // next panel width
        T *akk = a + k * ld + k;
        T *a12 = akk + b, *a21 = akk + b * ld, *a22 = akk + b * ld + b;
        // C <- L_B^{-1} P_B C (block row) and D <- D U_B^{-1} (column below)
        HIP_TRY(trsm_pair<T>(akk, ld, b, a12, ld, r, Linv(step), f->pivot ? f->piv + k : nullptr,
                             k, a21, ld, r, Uinv(step), abort, s0));
        HIP_TRY(Prec<T>::gemm(kGemmUpdate, r, bn, b, T(-1), a21, ld, a12, ld, T(1), a22, ld, abort,
                              s0));
        HIP_TRY(hipEventRecord(f->ev_narrow, s0));
        HIP_TRY(hipStreamWaitEvent(s1, f->ev_narrow, 0));
        HIP_TRY(factor_pivot_block<T>(f, a22, bn, k + b, Linv(step + 1), Uinv(step + 1), s1));
        HIP_TRY(hipEventRecord(f->ev_panel, s1));
        const bool bf16_upd = sizeof(T) == 4 && f->u16 != nullptr &&
                              (f->upd_terms == 1 || r >= kSplitUpdateMin);
        // columns bn .. bn + wm - 1 on the main stream, the last wa on the reserved units
        const int64_t wa = (r > bn && !bf16_upd) ? aux_columns<T>(f, r, r - bn, b) : 0;
        const int64_t wm = r - bn - wa;
        if (wa > 0) {
            HIP_TRY(hipStreamWaitEvent(f->aux, f->ev_panel, 0));
            HIP_TRY(Prec<T>::gemm(kGemmUpdate, r, wa, b, T(-1), a21, ld, a12 + bn + wm, ld, T(1),
                                  a22 + bn + wm, ld, abort, f->aux));
            HIP_TRY(hipEventRecord(f->ev_aux, f->aux));
            aux_pending = true;
        }
        const bool timed = wm > 0 && 2 * step + 1 < static_cast<int64_t>(f->upd_ev.size());
        if (timed) {
            HIP_TRY(hipEventRecord(f->upd_ev[2 * step], s0));
            f->upd_flops += 2.0 * static_cast<double>(r) * static_cast<double>(wm) * b;
        }
        if (wm > 0 && bf16_upd)
            HIP_TRY(update_bf16(f->upd_terms, r, wm, b, reinterpret_cast<const float *>(a21),
                                ld, reinterpret_cast<const float *>(a12 + bn), ld,
                                reinterpret_cast<float *>(a22 + bn), ld, f->u16, f->uldk,
                                f->urows, abort, s0));
        else if (wm > 0)
            HIP_TRY(Prec<T>::gemm(kGemmUpdate, r, wm, b, T(-1), a21, ld, a12 + bn, ld, T(1),
                                  a22 + bn, ld, abort, s0));
        if (timed) HIP_TRY(hipEventRecord(f->upd_ev[2 * step + 1], s0));
    }
    if (aux_pending) HIP_TRY(hipStreamWaitEvent(s0, f->ev_aux, 0));
    if (f->pivot) HIP_TRY(permute_left<T>(a, ld, n, nb, f->piv, abort, s0));
    if (f->main) {
        HIP_TRY(hipEventRecord(f->ev_join, s0));
        HIP_TRY(hipStreamWaitEvent(f->stream, f->ev_join, 0));
    }
    return hipSuccess;
}

// Draw the multiplier's parameters (and, for the FFT kinds, its spectrum).
template <typename T>
hipError_t draw_multiplier(rmge_factors *f) {
    const int64_t n = f->n;
    hipStream_t s = f->stream;
    switch (f->kind) {
    case RMGE_MULT_NONE: return hipSuccess;
    case RMGE_MULT_GAUSSIAN:
        // split16: the multiplier is the BF16-rounded draw (also used by the solves)
        if (f->split16 && n % 4 == 0)
            return normals_bf16t(reinterpret_cast<float *>(f->G), f->ht16, n, f->ldk16, f->seed,
                                 1, s);
        HIP_TRY(Prec<T>::normals(static_cast<T *>(f->G), n * n, f->seed, 1, s));
        if (f->split16)
            return round_h_bf16(reinterpret_cast<float *>(f->G), n, f->ht16, f->ldk16, s);
        return hipSuccess;
    default: {
        if (f->kind == RMGE_MULT_UNITARY_CIRCULANT) {
            // phases into the second half of params; with period m = n the
            // spectrum follows from them directly, else the first column goes
            // into the first half and is transformed like any circulant's
            HIP_TRY(launch_uniforms_f64(f->params + n, n, f->seed,
                                        static_cast<uint64_t>(f->kind), s));
            if (f->m == n) return unitary_spectrum(f->params + n, n, f->hhat, s);
            HIP_TRY(unitary_column(f->params + n, n, f->params, s));
        } else {
            HIP_TRY(launch_normals_f64(f->params, f->kind == RMGE_MULT_CIRCULANT ? n : 2 * n - 1,
                                       f->seed, static_cast<uint64_t>(f->kind), s));
        }
        HIP_TRY(fft_embed(is_circulant(f->kind) ? RMGE_MULT_CIRCULANT : f->kind, f->params, n,
                          f->m, f->hker, s));
        return fft_spectrum(f->hker, f->m, f->tw, f->hhat, s);
    }
    }
}

// M = A H into f->lu (precision T): one dense product, or one FFT pass over the
// rows; max |M| (for the growth statistic) is accumulated into `absmax` by the
// same kernels when it is not null.
template <typename T>
hipError_t multiply(rmge_factors *f, double *absmax) {
    const int64_t n = f->n;
    hipStream_t s = f->stream;
    T *lu = static_cast<T *>(f->lu);
    switch (f->kind) {
    case RMGE_MULT_NONE:
        HIP_TRY((convert_2d<double, T>(f->A, f->lda, lu, f->ld, n, n, s)));
        return absmax ? abs_max<T>(lu, f->ld, n, absmax - 2, s) : hipSuccess;
    case RMGE_MULT_GAUSSIAN:
        if (f->split16)  // A split into two BF16 terms, H in BF16 (round_a, draw_multiplier)
            return gemm_bf16x2(n, n, round_up(n, 32), f->a16, f->a16 + f->rows16 * f->ldk16,
                               f->ldk16, f->ht16, f->ldk16, reinterpret_cast<float *>(lu), f->ld,
                               s, absmax);
        if (f->a32)  // A already rounded to FP32 (round_a): an FP32 x FP32 product
            return gemm_f32(kGemmProduct, n, n, n, 1.0f, f->a32, f->ld,
                            static_cast<const float *>(f->G), n, 0.0f,
                            reinterpret_cast<float *>(lu), f->ld, nullptr, s, absmax);
        return Prec<T>::gemm_a64(n, n, n, f->A, f->lda, static_cast<const T *>(f->G), n, lu,
                                 f->ld, absmax, s);
    default:
        return fft_rows<double, T>(f->A, f->lda, 1, n, n, f->m, f->tw, f->hhat, 1, 0.0, lu, f->ld,
                                   1, s, absmax);
    }
}

// FP32 factors with a dense multiplier: round A to FP32 once (the same
// rounding the product would apply on load), so the product streams half the
// bytes for A.
hipError_t round_a(rmge_factors *f) {
    if (f->split16)
        return split_bf16(f->A, f->lda, f->n, f->a16, f->a16 + f->rows16 * f->ldk16, f->ldk16,
                          f->stream);
    if (!f->a32) return hipSuccess;
    return convert_2d<double, float>(f->A, f->lda, f->a32, f->ld, f->n, f->n, f->stream);
}

template <typename T>
hipError_t precondition(rmge_factors *f) {
    HIP_TRY(draw_multiplier<T>(f));
    HIP_TRY(round_a(f));
    return multiply<T>(f, nullptr);
}

template <typename T>
rmge_status run_factor(rmge_factors *f) {
    hipStream_t s = f->stream;
    f->stats_done = false;
    f->anorm_done = false;
    f->anorm1_done = false;
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(1), 0, s, f->st, f->scal);
    RMGE_TRY(hipGetLastError());
    RMGE_TRY(hipEventRecord(f->ev[0], s));
    RMGE_TRY(draw_multiplier<T>(f));
    RMGE_TRY(round_a(f));
    RMGE_TRY(hipEventRecord(f->ev[1], s));
    RMGE_TRY(multiply<T>(f, f->scal + 2));
    RMGE_TRY(hipEventRecord(f->ev[2], s));
    RMGE_TRY(hipEventRecord(f->ev[3], s));
    if (f->pivot) RMGE_TRY(iota(f->piv, f->n, s));
    f->upd_flops = 0.0;
    RMGE_TRY(genp_blocked<T>(f));
    RMGE_TRY(hipEventRecord(f->ev[4], s));
    {
        T *sl = static_cast<T *>(f->sinv);
        RMGE_TRY(diag_inverses<T>(static_cast<const T *>(f->lu), f->ld, f->n, sl,
                                  sl + f->sinv_rows * kSub, f->st, s));
        f->binv_done = false;  // the 128-row block inverses wait for a one-RHS solve
    }
    RMGE_TRY(hipMemcpyAsync(&f->host_st, f->st, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    RMGE_TRY(hipStreamSynchronize(s));
    float t01 = 0.f, t12 = 0.f, t34 = 0.f;
    (void)hipEventElapsedTime(&t01, f->ev[0], f->ev[1]);
    (void)hipEventElapsedTime(&t12, f->ev[1], f->ev[2]);
    (void)hipEventElapsedTime(&t34, f->ev[3], f->ev[4]);
    f->stats.ms_multiplier = t01;
    f->stats.ms_product = t12;
    f->stats.ms_factor = t34;
    {  // the bulk updates: the pairs recorded in this factorization
        double ms = 0.0;
        const int64_t steps = (f->n + f->block - 1) / f->block;
        for (int64_t st = 0; st < steps && 2 * st + 1 < static_cast<int64_t>(f->upd_ev.size());
             ++st) {
            const int64_t k = st * f->block, b = std::min<int64_t>(f->block, f->n - k);
            const int64_t r = f->n - k - b, bn = std::min<int64_t>(r, f->block);
            if (r <= bn || f->host_st.code != 0) continue;
            float t = 0.f;
            if (hipEventElapsedTime(&t, f->upd_ev[2 * st], f->upd_ev[2 * st + 1]) == hipSuccess)
                ms += t;
        }
        f->ms_update = ms;
    }
    f->stats.info = f->host_st.code ? f->host_st.info : -1;
    f->stats.status = f->host_st.code;
    f->stats.block = f->block;
    if (f->host_st.code == 4) return RMGE_ZERO_PIVOT;
    if (f->host_st.code == 5) return RMGE_NONFINITE;
    if (f->host_st.code != 0) return RMGE_EDEVICE;  // a bounded wait inside a kernel gave up
    return RMGE_OK;
}

void free_handle(rmge_factors *f) {
    if (!f) return;
    void *ptrs[] = {f->lu, f->G, f->params, f->hker, f->hhat, f->tw, f->inv, f->sinv, f->binv,
                    f->piv, f->st, f->a32, f->a16, f->ht16, f->u16, f->wht, f->scal, f->wy, f->wx, f->wr,
                    f->wnorm, f->wt, f->wsync, f->kv, f->kb};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (hipEvent_t &e : f->ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : {f->ev_narrow, f->ev_panel, f->ev_fork, f->ev_join, f->ev_aux})
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : f->upd_ev)
        if (e) (void)hipEventDestroy(e);
    if (f->side) (void)hipStreamDestroy(f->side);
    if (f->main) (void)hipStreamDestroy(f->main);
    if (f->aux) (void)hipStreamDestroy(f->aux);
    delete f;
}

rmge_status alloc_handle(rmge_factors *f) {
    const int64_t n = f->n;
    const size_t es = elem_size(f->prec);
    RMGE_TRY(hipMalloc(&f->lu, es * static_cast<size_t>(n) * f->ld));
    if (f->kind == RMGE_MULT_GAUSSIAN) RMGE_TRY(hipMalloc(&f->G, es * static_cast<size_t>(n * n)));
    if (f->kind == RMGE_MULT_GAUSSIAN && f->prec == RMGE_F32 && !f->split16)
        RMGE_TRY(hipMalloc(&f->a32, sizeof(float) * static_cast<size_t>(n) * f->ld));
    if (f->split16) {  // zero padding to whole tiles and K chunks, written once
        f->rows16 = round_up(n, 256);
        f->ldk16 = round_up(n, 64);
        const size_t one = sizeof(uint16_t) * static_cast<size_t>(f->rows16) * f->ldk16;
        RMGE_TRY(hipMalloc(&f->a16, 2 * one));
        RMGE_TRY(hipMalloc(&f->ht16, one));
        RMGE_TRY(hipMemsetAsync(f->a16, 0, 2 * one, f->stream));
        RMGE_TRY(hipMemsetAsync(f->ht16, 0, one, f->stream));
        RMGE_TRY(hipMalloc(&f->wht, sizeof(double) * static_cast<size_t>(gemv_ht_blocks(n) * n)));
    }
    if (f->upd_terms) {
        f->urows = round_up(n, 256);
        f->uldk = round_up(f->block, 32);
        const size_t ubytes = 2 * f->upd_terms * sizeof(uint16_t) *
                              static_cast<size_t>(f->urows) * f->uldk;
        if (ubytes <= INT32_MAX) {  // else the updates stay in FP32 (32-bit buffer offsets)
            RMGE_TRY(hipMalloc(&f->u16, ubytes));
            RMGE_TRY(hipMemsetAsync(f->u16, 0, ubytes, f->stream));
        } else {
            f->upd_terms = 0;
        }
    }
    if (is_fft_kind(f->kind)) {
        const int L = f->m / 2;
        RMGE_TRY(hipMalloc(&f->params, sizeof(double) * static_cast<size_t>(2 * n)));
        RMGE_TRY(hipMalloc(&f->hker, sizeof(double) * static_cast<size_t>(f->m)));
        RMGE_TRY(hipMalloc(&f->hhat, sizeof(double) * 2 * static_cast<size_t>(L + 1)));
        RMGE_TRY(hipMalloc(&f->tw, sizeof(double) * 2 * static_cast<size_t>(L + 1)));
        RMGE_TRY(fft_twiddles(f->m, f->tw, f->stream));
    }
    const size_t inv_elems = 4 * kMaxBlock * kSub;  // two buffers of (Linv, Uinv)
    RMGE_TRY(hipMalloc(&f->inv, es * inv_elems));
    RMGE_TRY(hipMemsetAsync(f->inv, 0, es * inv_elems, f->stream));
    f->sinv_rows = round_up(n, 256);
    const size_t sinv_elems = 2 * static_cast<size_t>(f->sinv_rows) * kSub;
    RMGE_TRY(hipMalloc(&f->sinv, es * sinv_elems));
    RMGE_TRY(hipMemsetAsync(f->sinv, 0, es * sinv_elems, f->stream));
    f->binv_rows = round_up(n, 128);
    RMGE_TRY(hipMalloc(&f->binv, sizeof(double) * 4 * static_cast<size_t>(f->binv_rows) * 128));
    if (f->pivot) RMGE_TRY(hipMalloc(&f->piv, sizeof(int) * static_cast<size_t>(n)));
    RMGE_TRY(hipMalloc(&f->st, sizeof(DevStatus)));
    RMGE_TRY(hipMalloc(&f->scal, sizeof(double) * 8));
    for (hipEvent_t &e : f->ev) RMGE_TRY(hipEventCreate(&e));
    // Look-ahead stream: kSideCUs compute units reserved for it, the rest for an
    // internal main stream (CU masks, same priority); RMGE_SIDE_CUS overrides
    // the count (0: no reservation, one shared pool).
    int side_cus = kSideCUs;
    if (const char *env = std::getenv("RMGE_SIDE_CUS")) side_cus = std::atoi(env);
    int dev = 0, ncu = 0;
    RMGE_TRY(hipGetDevice(&dev));
    RMGE_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    if (side_cus > 0 && side_cus < ncu) {
        std::vector<uint32_t> ms((ncu + 31) / 32, 0u), mm((ncu + 31) / 32, 0u);
        for (int c = 0; c < ncu; ++c) (c < side_cus ? ms : mm)[c / 32] |= 1u << (c % 32);
        RMGE_TRY(hipExtStreamCreateWithCUMask(&f->side, static_cast<uint32_t>(ms.size()), ms.data()));
        RMGE_TRY(hipExtStreamCreateWithCUMask(&f->main, static_cast<uint32_t>(mm.size()), mm.data()));
        RMGE_TRY(hipExtStreamCreateWithCUMask(&f->aux, static_cast<uint32_t>(ms.size()), ms.data()));
        RMGE_TRY(hipEventCreateWithFlags(&f->ev_aux, hipEventDisableTiming));
        f->cus_side = side_cus;
        f->cus_main = ncu - side_cus;
        f->aux_scale = 1.0;  // RMGE_AUX_SCALE overrides (0: the main stream does every update)
        if (const char *env = std::getenv("RMGE_AUX_SCALE")) f->aux_scale = std::atof(env);
    } else {
        RMGE_TRY(hipStreamCreateWithFlags(&f->side, hipStreamNonBlocking));
    }
    for (hipEvent_t *e : {&f->ev_narrow, &f->ev_panel, &f->ev_fork, &f->ev_join})
        RMGE_TRY(hipEventCreateWithFlags(e, hipEventDisableTiming));
    const int64_t steps = (n + f->block - 1) / f->block;
    if (steps <= kUpdEvents) {
        f->upd_ev.assign(static_cast<size_t>(2 * steps), nullptr);
        for (hipEvent_t &e : f->upd_ev) RMGE_TRY(hipEventCreate(&e));
    }
    return RMGE_OK;
}

// ------------------------------------------------------------------- solve

rmge_status ensure_solve_ws(rmge_factors *f, int64_t nrhs, bool need_t) {
    const int64_t n = f->n;
    if (nrhs > f->ws_nrhs) {
        for (double **p : {&f->wy, &f->wx}) {
            if (*p) (void)hipFree(*p);
            *p = nullptr;
        }
        if (f->wr) (void)hipFree(f->wr);
        if (f->wnorm) (void)hipFree(f->wnorm);
        f->wr = f->wnorm = nullptr;
        f->ws_nrhs = 0;
        RMGE_TRY(hipMalloc(&f->wy, sizeof(double) * static_cast<size_t>(n * nrhs)));
        RMGE_TRY(hipMalloc(&f->wx, sizeof(double) * static_cast<size_t>(n * nrhs)));
        RMGE_TRY(hipMalloc(&f->wr, sizeof(double) * static_cast<size_t>(n * nrhs)));
        RMGE_TRY(hipMalloc(&f->wnorm, sizeof(double) * static_cast<size_t>(4 * nrhs + 8)));
        f->ws_nrhs = nrhs;
    }
    if (!f->wsync) {
        RMGE_TRY(hipMalloc(&f->wsync, sizeof(int) * 2));
        RMGE_TRY(hipMemsetAsync(f->wsync, 0, sizeof(int) * 2, f->stream));
    }
    if (need_t) {
        const int64_t want = ((n + 255) / 256) * n * (nrhs < 16 ? nrhs : 16);
        if (want > f->wt_size) {
            if (f->wt) (void)hipFree(f->wt);
            f->wt = nullptr;
            f->wt_size = 0;
            RMGE_TRY(hipMalloc(&f->wt, sizeof(double) * static_cast<size_t>(want)));
            f->wt_size = want;
        }
    }
    return RMGE_OK;
}

// Triangular solves on the workspace: wy (FP64, n x nrhs) <- U^{-1} L^{-1} wy
// (`adjoint`: U^{-T} then L^{-T}), one persistent launch per solve and group
// of 16 right-hand sides, through wx.
template <typename T>
hipError_t tri_solves(rmge_factors *f, int64_t nrhs, bool adjoint) {
    const int64_t n = f->n, ld = f->ld;
    const T *lu = static_cast<const T *>(f->lu);
    double *Y = f->wy, *X = f->wx;
    const T *Linv = static_cast<const T *>(f->sinv), *Uinv = Linv + f->sinv_rows * kSub;
    hipStream_t s = f->stream;
    // L then U (solve), or U^T then L^T (adjoint)
    const int first = adjoint ? 2 : 0, second = adjoint ? 3 : 1;
    const T *dfirst = adjoint ? Uinv : Linv, *dsecond = adjoint ? Linv : Uinv;
    if (nrhs == 1 && !adjoint) {  // 128-row blocks with the FP64 block inverses
        const int64_t part = f->binv_rows * 128;
        if (!f->binv_done) {  // once per factorization, in stream order after it
            HIP_TRY(block_inverses128<T>(lu, ld, n, f->binv, f->binv + part, f->binv + 2 * part,
                                         f->binv + 3 * part, s));
            f->binv_done = true;
        }
        const double *bl = f->binv, *bu = bl + part, *wl = bl + 2 * part, *wu = bl + 3 * part;
        HIP_TRY(trsv128<T>(0, lu, ld, n, bl, wl, Y, X, 1, f->wsync, s));
        return trsv128<T>(1, lu, ld, n, bu, wu, X, Y, 1, f->wsync, s);
    }
    for (int64_t g = 0; g < nrhs; g += 16) {
        const int nr = static_cast<int>((nrhs - g) < 16 ? (nrhs - g) : 16);
        HIP_TRY(trsv_full<T>(first, lu, ld, n, dfirst, Y + g, X + g, nrhs, nr, f->wsync, s));
        HIP_TRY(trsv_full<T>(second, lu, ld, n, dsecond, X + g, Y + g, nrhs, nr, f->wsync, s));
    }
    return hipSuccess;
}

// After a stream sync: did a persistent solve give up waiting?
rmge_status solve_sync_error(rmge_factors *f) {
    int err = 0;
    RMGE_TRY(hipMemcpy(&err, f->wsync + 1, sizeof(int), hipMemcpyDeviceToHost));
    if (err) {
        RMGE_TRY(hipMemset(f->wsync + 1, 0, sizeof(int)));
        return RMGE_EDEVICE;
    }
    return RMGE_OK;
}

// X = beta X + H U^{-1} L^{-1} P src   (src FP64 n x nrhs, lds; P = I unless pivoted)
template <typename T>
hipError_t apply_inverse(rmge_factors *f, const double *src, int64_t lds, int64_t nrhs, double *X,
                         int64_t ldx, double beta) {
    const int64_t n = f->n;
    hipStream_t s = f->stream;
    double *Y = f->wy;
    hipError_t e = convert_2d<double, double>(src, lds, Y, nrhs, n, nrhs, s,
                                              f->pivot ? f->piv : nullptr);
    if (e != hipSuccess) return e;
    if ((e = tri_solves<T>(f, nrhs, false)) != hipSuccess) return e;
    switch (f->kind) {
    case RMGE_MULT_NONE:
        return axpby_2d<double>(Y, nrhs, X, ldx, n, static_cast<int>(nrhs), beta, s);
    case RMGE_MULT_GAUSSIAN:
        // split16: the BF16 copy of H (exact, half the bytes of the FP32 one)
        if (f->split16 && nrhs == 1)
            return gemv_ht(n, f->ht16, f->ldk16, Y, 1, beta, X, ldx, f->wht, s);
        for (int64_t g = 0; g < nrhs; g += 16) {
            const int nr = static_cast<int>((nrhs - g) < 16 ? (nrhs - g) : 16);
            e = gemv_n<T, double, double>(n, n, 1.0, static_cast<const T *>(f->G), n, Y + g,
                                          nrhs, beta, X + g, ldx, nr, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    default:
        return fft_rows<double, double>(Y, 1, nrhs, nrhs, n, f->m, f->tw, f->hhat, 0, beta, X, 1,
                                        ldx, s);
    }
}

// R = B - A X; returns eta = max_r ||R_r||_inf / (||A||_inf ||X_r||_inf + ||B_r||_inf).
rmge_status residual_eta(rmge_factors *f, const double *B, int64_t ldb, int64_t nrhs,
                         const double *X, int64_t ldx, double *eta) {
    const int64_t n = f->n;
    hipStream_t s = f->stream;
    double *R = f->wr, *nrm = f->wnorm;
    RMGE_TRY((convert_2d<double, double>(B, ldb, R, nrhs, n, nrhs, s)));
    // ||A||_inf, once per factorization: from the residual's own reads of A
    // when its product takes at most four right-hand sides, else a pass of its own
    const bool fuse_norm = !f->anorm_done && nrhs <= 4;
    if (!f->anorm_done) RMGE_TRY(fill_f64(f->scal + 3, 1, 0.0, s));
    for (int64_t g = 0; g < nrhs; g += 16) {
        const int nr = static_cast<int>((nrhs - g) < 16 ? (nrhs - g) : 16);
        RMGE_TRY((gemv_n<double, double, double>(n, n, -1.0, f->A, f->lda, X + g, ldx, 1.0, R + g,
                                                 nrhs, nr, s, fuse_norm ? f->scal + 3 : nullptr)));
    }
    RMGE_TRY(fill_f64(nrm, 3 * nrhs, 0.0, s));
    RMGE_TRY(colmax_abs(R, nrhs, n, static_cast<int>(nrhs), nrm, s));
    RMGE_TRY(colmax_abs(X, ldx, n, static_cast<int>(nrhs), nrm + nrhs, s));
    RMGE_TRY(colmax_abs(B, ldb, n, static_cast<int>(nrhs), nrm + 2 * nrhs, s));
    if (!f->anorm_done && !fuse_norm) RMGE_TRY(norm_inf(f->A, f->lda, n, f->scal + 3, s));
    std::vector<double> h(static_cast<size_t>(3 * nrhs));
    RMGE_TRY(hipMemcpyAsync(h.data(), nrm, sizeof(double) * 3 * nrhs, hipMemcpyDeviceToHost, s));
    if (!f->anorm_done)
        RMGE_TRY(hipMemcpyAsync(&f->anorm, f->scal + 3, sizeof(double), hipMemcpyDeviceToHost, s));
    RMGE_TRY(hipStreamSynchronize(s));
    f->anorm_done = true;
    double worst = 0.0;
    for (int64_t r = 0; r < nrhs; ++r) {
        const double e = h[r] / (f->anorm * h[nrhs + r] + h[2 * nrhs + r]);
        if (e > worst || e != e) worst = e;
    }
    *eta = worst;
    return RMGE_OK;
}

template <typename T>
rmge_status run_solve(rmge_factors *f, const double *B, int64_t nrhs, int64_t ldb, double *X,
                      int64_t ldx, int32_t max_refine, double tol, rmge_solve_stats *st) {
    rmge_status rs = ensure_solve_ws(f, nrhs, false);
    if (rs != RMGE_OK) return rs;
    RMGE_TRY(apply_inverse<T>(f, B, ldb, nrhs, X, ldx, 0.0));
    double eta = 0.0;
    rs = residual_eta(f, B, ldb, nrhs, X, ldx, &eta);
    if (rs != RMGE_OK) return rs;
    rmge_solve_stats loc{};
    loc.eta0 = eta;
    loc.eta_hist[0] = eta;
    int it = 0;
    while (it < max_refine && !(tol > 0.0 && eta <= tol)) {
        RMGE_TRY(apply_inverse<T>(f, f->wr, nrhs, nrhs, X, ldx, 1.0));
        ++it;
        rs = residual_eta(f, B, ldb, nrhs, X, ldx, &eta);
        if (rs != RMGE_OK) return rs;
        loc.eta_hist[it] = eta;
    }
    rs = solve_sync_error(f);
    if (rs != RMGE_OK) return rs;
    loc.iters = it;
    loc.eta = eta;
    loc.converged = (tol <= 0.0 || eta <= tol) ? 1 : 0;
    if (st) *st = loc;
    return loc.converged ? RMGE_OK : RMGE_NOT_CONVERGED;
}

// Y = beta Y + P^T L^{-T} U^{-T} H^T src   (src FP64 n x nrhs, lds)
template <typename T>
hipError_t apply_adjoint(rmge_factors *f, const double *src, int64_t lds, int64_t nrhs,
                         double *Y, int64_t ldy, double beta) {
    const int64_t n = f->n;
    hipStream_t s = f->stream;
    double *Z = f->wy;
    switch (f->kind) {
    case RMGE_MULT_NONE:
        HIP_TRY((convert_2d<double, double>(src, lds, Z, nrhs, n, nrhs, s)));
        break;
    case RMGE_MULT_GAUSSIAN:
        for (int64_t g = 0; g < nrhs; g += 16) {
            const int nr = static_cast<int>((nrhs - g) < 16 ? (nrhs - g) : 16);
            HIP_TRY((gemv_t<T, double, double>(n, n, static_cast<const T *>(f->G), n, src + g, lds,
                                               Z + g, nrhs, nr, f->wt, s)));
        }
        break;
    default:
        HIP_TRY((fft_rows<double, double>(src, 1, lds, nrhs, n, f->m, f->tw, f->hhat, 1, 0.0, Z, 1,
                                          nrhs, s)));
    }
    HIP_TRY(tri_solves<T>(f, nrhs, true));
    // row t of the solution goes back to row piv[t]
    return axpby_2d<double>(Z, nrhs, Y, ldy, n, static_cast<int>(nrhs), beta, s,
                            f->pivot ? f->piv : nullptr);
}

// R = W - A^T Y; eta = max_r ||R_r||_inf / (||A^T||_inf ||Y_r||_inf + ||W_r||_inf).
rmge_status adjoint_residual_eta(rmge_factors *f, const double *W, int64_t ldw, int64_t nrhs,
                                 const double *Y, int64_t ldy, double *eta) {
    const int64_t n = f->n;
    hipStream_t s = f->stream;
    double *R = f->wr, *nrm = f->wnorm;
    for (int64_t g = 0; g < nrhs; g += 16) {
        const int nr = static_cast<int>((nrhs - g) < 16 ? (nrhs - g) : 16);
        RMGE_TRY((gemv_t<double, double, double>(n, n, f->A, f->lda, Y + g, ldy, R + g, nrhs, nr,
                                                 f->wt, s)));
    }
    RMGE_TRY(axpby_2d<double>(W, ldw, R, nrhs, n, static_cast<int>(nrhs), -1.0, s));
    RMGE_TRY(fill_f64(nrm, 3 * nrhs, 0.0, s));
    RMGE_TRY(colmax_abs(R, nrhs, n, static_cast<int>(nrhs), nrm, s));
    RMGE_TRY(colmax_abs(Y, ldy, n, static_cast<int>(nrhs), nrm + nrhs, s));
    RMGE_TRY(colmax_abs(W, ldw, n, static_cast<int>(nrhs), nrm + 2 * nrhs, s));
    if (!f->anorm1_done) {
        RMGE_TRY(fill_f64(f->scal + 4, 1, 0.0, s));
        RMGE_TRY(norm_one(f->A, f->lda, n, f->wt, f->scal + 4, s));
    }
    std::vector<double> h(static_cast<size_t>(3 * nrhs));
    RMGE_TRY(hipMemcpyAsync(h.data(), nrm, sizeof(double) * 3 * nrhs, hipMemcpyDeviceToHost, s));
    if (!f->anorm1_done)
        RMGE_TRY(hipMemcpyAsync(&f->anorm1, f->scal + 4, sizeof(double), hipMemcpyDeviceToHost, s));
    RMGE_TRY(hipStreamSynchronize(s));
    f->anorm1_done = true;
    double worst = 0.0;
    for (int64_t r = 0; r < nrhs; ++r) {
        const double e = h[r] / (f->anorm1 * h[nrhs + r] + h[2 * nrhs + r]);
        if (e > worst || e != e) worst = e;
    }
    *eta = worst;
    return RMGE_OK;
}

template <typename T>
rmge_status run_adjoint(rmge_factors *f, const double *W, int64_t nrhs, int64_t ldw, double *Y,
                        int64_t ldy, int32_t max_refine, double tol, rmge_solve_stats *st) {
    rmge_status rs = ensure_solve_ws(f, nrhs, true);
    if (rs != RMGE_OK) return rs;
    RMGE_TRY(apply_adjoint<T>(f, W, ldw, nrhs, Y, ldy, 0.0));
    if (!st && max_refine == 0) {  // plain adjoint application
        RMGE_TRY(hipStreamSynchronize(f->stream));
        return solve_sync_error(f);
    }
    double eta = 0.0;
    if ((rs = adjoint_residual_eta(f, W, ldw, nrhs, Y, ldy, &eta)) != RMGE_OK) return rs;
    rmge_solve_stats loc{};
    loc.eta0 = eta;
    loc.eta_hist[0] = eta;
    int it = 0;
    while (it < max_refine && !(tol > 0.0 && eta <= tol)) {
        RMGE_TRY(apply_adjoint<T>(f, f->wr, nrhs, nrhs, Y, ldy, 1.0));
        ++it;
        if ((rs = adjoint_residual_eta(f, W, ldw, nrhs, Y, ldy, &eta)) != RMGE_OK) return rs;
        loc.eta_hist[it] = eta;
    }
    if ((rs = solve_sync_error(f)) != RMGE_OK) return rs;
    loc.iters = it;
    loc.eta = eta;
    loc.converged = (tol <= 0.0 || eta <= tol) ? 1 : 0;
    if (st) *st = loc;
    return loc.converged ? RMGE_OK : RMGE_NOT_CONVERGED;
}

// ------------------------------------------------------------- GMRES-IR
//
// Refinement by restarted flexible GMRES, right-preconditioned by the
// factors: for each right-hand side, outer steps r = b - A x (FP64), inner
// Krylov iterations on A d = r with z_j = H U^{-1} L^{-1} P v_j (the same
// application of the preprocessed inverse as one classical refinement step),
// w = A z_j, classical Gram-Schmidt applied twice, Givens rotations on the
// host; then x += Z y.  The transposed system A^T y = w runs the same way with
// A^T and the adjoint application P^T L^{-T} U^{-T} H^T.  The FP64 basis makes the iteration converge when the
// factors are too inaccurate for classical refinement to contract (large
// growth, or kappa(A H) u_factor near 1).

constexpr int kMaxRestart = 64;

rmge_status ensure_krylov_ws(rmge_factors *f, int restart) {
    if (f->kv && f->kv_restart >= restart) return RMGE_OK;
    if (f->kv) (void)hipFree(f->kv);
    f->kv = nullptr;
    f->kv_restart = 0;
    const size_t n = static_cast<size_t>(f->n);
    const size_t words = (2 * static_cast<size_t>(restart) + 2) * n + 256 * kMaxRestart +
                         6 * kMaxRestart;
    RMGE_TRY(hipMalloc(&f->kv, sizeof(double) * words));
    f->kv_restart = restart;
    return RMGE_OK;
}

// trans = 0: A x = b with the preconditioner H U^{-1} L^{-1} P;
// trans = 1: A^T y = w with the preconditioner P^T L^{-T} U^{-T} H^T.
template <typename T>
rmge_status run_gmres(rmge_factors *f, bool trans, const double *B, int64_t nrhs, int64_t ldb,
                      double *X, int64_t ldx, int32_t max_iters, int32_t restart, double tol,
                      rmge_solve_stats *st) {
    rmge_status rs = ensure_solve_ws(f, nrhs, trans);
    if (rs != RMGE_OK) return rs;
    if ((rs = ensure_krylov_ws(f, restart)) != RMGE_OK) return rs;
    const int64_t n = f->n;
    hipStream_t s = f->stream;
    double *V = f->kv;                             // (restart + 1) x n
    double *Z = V + (restart + 1) * n;             // restart x n
    double *R = Z + restart * n;                   // n
    double *part = R + n;                          // 256 x kMaxRestart
    double *dv = part + 256 * kMaxRestart;         // [0, 64) h, [64, 128) h2, [128] |w|^2,
                                                   // [129 ..] norms; [192, 256) y
    double *hy = dv + 3 * kMaxRestart;
    double *rc = dv + 4 * kMaxRestart;             // residual coefficients (restart + 1)
    auto precond = [&](const double *src, int64_t lds, int64_t nr, double *dst, int64_t ldd) {
        return trans ? apply_adjoint<T>(f, src, lds, nr, dst, ldd, 0.0)
                     : apply_inverse<T>(f, src, lds, nr, dst, ldd, 0.0);
    };
    // dst = op(A) z for one vector, op(A) = A or A^T
    auto op = [&](const double *z, int64_t ldz, double *dst) -> hipError_t {
        if (trans)
            return gemv_t<double, double, double>(n, n, f->A, f->lda, z, ldz, dst, 1, 1, f->wt,
                                                  s);
        return gemv_n<double, double, double>(n, n, 1.0, f->A, f->lda, z, ldz, 0.0, dst, 1, 1, s);
    };
    // initial solve for every right-hand side (one classical application)
    RMGE_TRY(precond(B, ldb, nrhs, X, ldx));
    double anorm = 0.0;
    if (!trans) {
        if (!f->anorm_done) {
            RMGE_TRY(fill_f64(f->scal + 3, 1, 0.0, s));
            RMGE_TRY(norm_inf(f->A, f->lda, n, f->scal + 3, s));
            RMGE_TRY(hipMemcpyAsync(&f->anorm, f->scal + 3, sizeof(double), hipMemcpyDeviceToHost,
                                    s));
            RMGE_TRY(hipStreamSynchronize(s));
            f->anorm_done = true;
        }
        anorm = f->anorm;
    } else {
        if (!f->anorm1_done) {
            RMGE_TRY(fill_f64(f->scal + 4, 1, 0.0, s));
            RMGE_TRY(norm_one(f->A, f->lda, n, f->wt, f->scal + 4, s));
            RMGE_TRY(hipMemcpyAsync(&f->anorm1, f->scal + 4, sizeof(double),
                                    hipMemcpyDeviceToHost, s));
            RMGE_TRY(hipStreamSynchronize(s));
            f->anorm1_done = true;
        }
        anorm = f->anorm1;
    }
    rmge_solve_stats loc{};
    int hist = 0, total = 0;
    bool all_ok = true;
    double worst0 = 0.0, worst = 0.0;
    std::vector<double> H(static_cast<size_t>((restart + 1) * restart)), cs(restart), sn(restart),
        g(restart + 1), y(restart), hh(3 * kMaxRestart), u(restart + 1);
    const double sqrt_n = std::sqrt(static_cast<double>(n));
    for (int64_t c = 0; c < nrhs; ++c) {
        double eta = 0.0;
        bool first = true;
        int used = 0;  // inner iterations spent on this right-hand side
        while (true) {
            // r = b - op(A) x, eta, ||r||_2
            RMGE_TRY(op(X + c, ldx, R));
            RMGE_TRY(axpby_2d<double>(B + c, ldb, R, 1, n, 1, -1.0, s));
            RMGE_TRY(fill_f64(dv + 129, 3, 0.0, s));
            RMGE_TRY(colmax_abs(R, 1, n, 1, dv + 129, s));
            RMGE_TRY(colmax_abs(X + c, ldx, n, 1, dv + 130, s));
            RMGE_TRY(colmax_abs(B + c, ldb, n, 1, dv + 131, s));
            RMGE_TRY(mdot(R, n, 1, R, part, dv + 128, false, s));
            RMGE_TRY(hipMemcpyAsync(hh.data() + 128, dv + 128, 4 * sizeof(double),
                                    hipMemcpyDeviceToHost, s));
            RMGE_TRY(hipStreamSynchronize(s));
            const double rinf = hh[129], xinf = hh[130], binf = hh[131];
            const double scale = anorm * xinf + binf;
            eta = rinf / scale;
            if (first) {
                worst0 = (eta > worst0 || eta != eta) ? eta : worst0;
                first = false;
            }
            if (hist < 17) loc.eta_hist[hist++] = eta;
            if (!(eta > tol) || used >= max_iters || eta != eta) break;
            const double beta = std::sqrt(hh[128]);
            if (!(beta > 0.0)) break;
            const double target = 0.5 * tol * scale;  // ||r||_2 <= target => eta <= tol / 2
            RMGE_TRY(scale_copy(V, R, 1, n, 1.0 / beta, s));
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = beta;
            int k = 0;
            for (int j = 0; j < restart && used < max_iters; ++j) {
                double *vj = V + j * n, *w = V + (j + 1) * n, *zj = Z + j * n;
                RMGE_TRY(precond(vj, 1, 1, zj, 1));
                RMGE_TRY(op(zj, 1, w));
                RMGE_TRY(mdot(V, n, j + 1, w, part, dv, false, s));
                RMGE_TRY(lincomb(w, 1, V, n, j + 1, dv, -1.0, s));
                RMGE_TRY(mdot(V, n, j + 1, w, part, dv + kMaxRestart, false, s));
                RMGE_TRY(lincomb(w, 1, V, n, j + 1, dv + kMaxRestart, -1.0, s));
                RMGE_TRY(mdot(w, n, 1, w, part, dv + 2 * kMaxRestart, false, s));
                RMGE_TRY(hipMemcpyAsync(hh.data(), dv, (2 * kMaxRestart + 1) * sizeof(double),
                                        hipMemcpyDeviceToHost, s));
                RMGE_TRY(hipStreamSynchronize(s));
                ++total;
                ++used;
                double *col = H.data() + static_cast<size_t>(j) * (restart + 1);
                for (int i = 0; i <= j; ++i) col[i] = hh[i] + hh[kMaxRestart + i];
                const double hnext = std::sqrt(hh[2 * kMaxRestart]);
                col[j + 1] = hnext;
                if (hnext > 0.0) RMGE_TRY(scale_copy(w, w, 1, n, 1.0 / hnext, s));
                for (int i = 0; i < j; ++i) {  // earlier rotations
                    const double a = col[i], b = col[i + 1];
                    col[i] = cs[i] * a + sn[i] * b;
                    col[i + 1] = -sn[i] * a + cs[i] * b;
                }
                const double a = col[j], b = col[j + 1];
                const double rr = std::hypot(a, b);
                cs[j] = rr > 0.0 ? a / rr : 1.0;
                sn[j] = rr > 0.0 ? b / rr : 0.0;
                col[j] = rr;
                col[j + 1] = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
                k = j + 1;
                const double rn2 = std::fabs(g[j + 1]);
                if (rn2 <= target || !(hnext > 1e-300 * beta)) break;
                if (rn2 <= sqrt_n * target && j + 1 < restart) {
                    // ||r||_inf may already meet the target: form the residual
                    // from the basis, r = g_{j+1} V_{0..j+1} (G_0^T .. G_j^T e_{j+1}),
                    // and stop when its max norm does (the outer step then checks
                    // b - op(A) x itself; the last step of a cycle goes there anyway)
                    std::fill(u.begin(), u.begin() + (j + 2), 0.0);
                    u[j + 1] = g[j + 1];
                    for (int i = j; i >= 0; --i) {
                        const double a0 = u[i], b0 = u[i + 1];
                        u[i] = cs[i] * a0 - sn[i] * b0;
                        u[i + 1] = sn[i] * a0 + cs[i] * b0;
                    }
                    RMGE_TRY(hipMemcpyAsync(rc, u.data(), (j + 2) * sizeof(double),
                                            hipMemcpyHostToDevice, s));
                    RMGE_TRY(fill_f64(R, n, 0.0, s));
                    RMGE_TRY(lincomb(R, 1, V, n, j + 2, rc, 1.0, s));
                    RMGE_TRY(fill_f64(dv + 129, 1, 0.0, s));
                    RMGE_TRY(colmax_abs(R, 1, n, 1, dv + 129, s));
                    RMGE_TRY(hipMemcpyAsync(hh.data() + 129, dv + 129, sizeof(double),
                                            hipMemcpyDeviceToHost, s));
                    RMGE_TRY(hipStreamSynchronize(s));
                    if (hh[129] <= target) break;
                }
            }
            if (k == 0) break;
            for (int i = k - 1; i >= 0; --i) {  // R y = g
                double t = g[i];
                for (int l = i + 1; l < k; ++l) t -= H[static_cast<size_t>(l) * (restart + 1) + i] * y[l];
                const double d = H[static_cast<size_t>(i) * (restart + 1) + i];
                y[i] = d != 0.0 ? t / d : 0.0;
            }
            RMGE_TRY(hipMemcpyAsync(hy, y.data(), k * sizeof(double), hipMemcpyHostToDevice, s));
            RMGE_TRY(lincomb(X + c, ldx, Z, n, k, hy, 1.0, s));
        }
        worst = (eta > worst || eta != eta) ? eta : worst;
        if (!(eta <= tol)) all_ok = false;
    }
    rs = solve_sync_error(f);
    if (rs != RMGE_OK) return rs;
    loc.iters = total;
    loc.eta0 = worst0;
    loc.eta = worst;
    loc.converged = all_ok ? 1 : 0;
    if (st) *st = loc;
    return all_ok ? RMGE_OK : RMGE_NOT_CONVERGED;
}

// Several right-hand sides at once (2 <= nrhs <= 64): the same restarted FGMRES
// as run_gmres for every column, with the columns' Arnoldi processes advanced
// together, so each iteration is one preconditioner application, one product
// with op(A) and one Gram-Schmidt pass for all of them, and one host
// synchronisation (for the columns' Givens rotations) instead of one per
// column.  A column that has met the tolerance, or whose Krylov space stopped
// growing, keeps its iterate: its basis vectors from then on are zero.
template <typename T>
rmge_status run_gmres_block(rmge_factors *f, bool trans, const double *B, int64_t m, int64_t ldb,
                            double *X, int64_t ldx, int32_t max_iters, int32_t restart, double tol,
                            rmge_solve_stats *st) {
    rmge_status rs = ensure_solve_ws(f, m, trans);
    if (rs != RMGE_OK) return rs;
    const int64_t n = f->n;
    const int R = restart;
    const int mi = static_cast<int>(m);
    const int64_t nm = n * m;
    const int64_t words = (2 * static_cast<int64_t>(R) + 2) * nm + 256 * (R + 1) * m +
                          (3 * static_cast<int64_t>(R) + 8) * m;
    if (f->kb_words < words) {
        if (f->kb) (void)hipFree(f->kb);
        f->kb = nullptr;
        f->kb_words = 0;
        RMGE_TRY(hipMalloc(&f->kb, sizeof(double) * static_cast<size_t>(words)));
        f->kb_words = words;
    }
    hipStream_t s = f->stream;
    double *V = f->kb;                         // (R + 1) blocks n x m
    double *Z = V + (R + 1) * nm;              // R blocks
    double *W = Z + R * nm;                    // n x m
    double *part = W + nm;                     // 256 (R + 1) m
    double *d1 = part + 256 * (R + 1) * m;     // (R + 1) m: first Gram-Schmidt pass
    double *d2 = d1 + (R + 1) * m;             // (R + 1) m: second pass
    double *w2 = d2 + (R + 1) * m;             // m
    double *scl = w2 + m;                      // m
    double *yv = scl + m;                      // R m: update coefficients
    double *nrm = yv + R * m;                  // 3 m: max norms of r, x, b
    auto precond = [&](const double *src, int64_t lds, double *dst, int64_t ldd) {
        return trans ? apply_adjoint<T>(f, src, lds, m, dst, ldd, 0.0)
                     : apply_inverse<T>(f, src, lds, m, dst, ldd, 0.0);
    };
    // dst (n x m, ld m) = op(A) z (ld ldz), sixteen columns a launch
    auto op = [&](const double *z, int64_t ldz, double *dst) -> hipError_t {
        for (int64_t g = 0; g < m; g += 16) {
            const int nr = static_cast<int>((m - g) < 16 ? (m - g) : 16);
            const hipError_t e =
                trans ? gemv_t<double, double, double>(n, n, f->A, f->lda, z + g, ldz, dst + g, m,
                                                       nr, f->wt, s)
                      : gemv_n<double, double, double>(n, n, 1.0, f->A, f->lda, z + g, ldz, 0.0,
                                                       dst + g, m, nr, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    RMGE_TRY(precond(B, ldb, X, ldx));
    double anorm = 0.0;
    {
        double *slot = trans ? f->scal + 4 : f->scal + 3;
        bool &done = trans ? f->anorm1_done : f->anorm_done;
        double &val = trans ? f->anorm1 : f->anorm;
        if (!done) {
            RMGE_TRY(fill_f64(slot, 1, 0.0, s));
            if (trans)
                RMGE_TRY(norm_one(f->A, f->lda, n, f->wt, slot, s));
            else
                RMGE_TRY(norm_inf(f->A, f->lda, n, slot, s));
            RMGE_TRY(hipMemcpyAsync(&val, slot, sizeof(double), hipMemcpyDeviceToHost, s));
            RMGE_TRY(hipStreamSynchronize(s));
            done = true;
        }
        anorm = val;
    }
    const size_t M = static_cast<size_t>(m);
    std::vector<double> H(M * (R + 1) * R), cs(M * R), sn(M * R), g(M * (R + 1)), hy(M * R),
        hh(M * (2 * (R + 1) + 1)), eta(M, 0.0), eta0(M, -1.0), tgt(M, 0.0), beta(M, 0.0),
        sc(M, 0.0), hn(M), hst(3 * M);
    std::vector<char> active(M, 0), live(M, 0);
    int hist = 0, total = 0;
    rmge_solve_stats loc{};
    while (true) {
        // W = B - op(A) X; per column eta and ||r||_2
        RMGE_TRY(op(X, ldx, W));
        RMGE_TRY((axpby_2d<double>(B, ldb, W, m, n, mi, -1.0, s)));
        RMGE_TRY(fill_f64(nrm, 3 * m, 0.0, s));
        RMGE_TRY(colmax_abs(W, m, n, mi, nrm, s));
        RMGE_TRY(colmax_abs(X, ldx, n, mi, nrm + m, s));
        RMGE_TRY(colmax_abs(B, ldb, n, mi, nrm + 2 * m, s));
        RMGE_TRY(bdot(W, n, mi, 1, W, m, part, w2, false, s));
        RMGE_TRY(hipMemcpyAsync(hst.data(), nrm, sizeof(double) * 3 * M, hipMemcpyDeviceToHost, s));
        RMGE_TRY(hipMemcpyAsync(hn.data(), w2, sizeof(double) * M, hipMemcpyDeviceToHost, s));
        RMGE_TRY(hipStreamSynchronize(s));
        double worst = 0.0;
        bool any = false;
        for (size_t c = 0; c < M; ++c) {
            const double scale = anorm * hst[M + c] + hst[2 * M + c];
            eta[c] = hst[c] / scale;
            if (eta0[c] < 0.0) eta0[c] = eta[c];
            worst = (eta[c] > worst || eta[c] != eta[c]) ? eta[c] : worst;
            beta[c] = std::sqrt(hn[c]);
            active[c] = (eta[c] > tol && eta[c] == eta[c] && beta[c] > 0.0) ? 1 : 0;
            tgt[c] = 0.5 * tol * scale;
            any = any || active[c];
        }
        if (hist < 17) loc.eta_hist[hist++] = worst;
        if (!any || total >= max_iters) break;
        // V_0 = W / beta on the active columns, zero elsewhere
        for (size_t c = 0; c < M; ++c) {
            sc[c] = active[c] ? 1.0 / beta[c] : 0.0;
            live[c] = active[c];
        }
        RMGE_TRY(hipMemcpyAsync(scl, sc.data(), sizeof(double) * M, hipMemcpyHostToDevice, s));
        RMGE_TRY(bscale(V, W, m, n, mi, scl, s));
        std::fill(g.begin(), g.end(), 0.0);
        for (size_t c = 0; c < M; ++c) g[c * (R + 1)] = active[c] ? beta[c] : 0.0;
        int k = 0;
        for (int j = 0; j < R && total < max_iters; ++j) {
            double *Vj = V + j * nm, *Zj = Z + j * nm, *Vn = V + (j + 1) * nm;
            RMGE_TRY(precond(Vj, m, Zj, m));
            RMGE_TRY(op(Zj, m, W));
            RMGE_TRY(bdot(V, n, mi, j + 1, W, m, part, d1, false, s));
            RMGE_TRY(blincomb(W, m, V, n, mi, j + 1, d1, -1.0, s));
            RMGE_TRY(bdot(V, n, mi, j + 1, W, m, part, d2, false, s));
            RMGE_TRY(blincomb(W, m, V, n, mi, j + 1, d2, -1.0, s));
            RMGE_TRY(bdot(W, n, mi, 1, W, m, part, w2, false, s));
            const size_t nd = static_cast<size_t>(j + 1) * M;
            RMGE_TRY(hipMemcpyAsync(hh.data(), d1, sizeof(double) * nd, hipMemcpyDeviceToHost, s));
            RMGE_TRY(hipMemcpyAsync(hh.data() + nd, d2, sizeof(double) * nd, hipMemcpyDeviceToHost,
                                    s));
            RMGE_TRY(hipMemcpyAsync(hn.data(), w2, sizeof(double) * M, hipMemcpyDeviceToHost, s));
            RMGE_TRY(hipStreamSynchronize(s));
            ++total;
            k = j + 1;
            bool more = false;
            for (size_t c = 0; c < M; ++c) {
                sc[c] = 0.0;
                if (!live[c]) continue;
                double *col = H.data() + (c * R + j) * (R + 1);
                for (int i = 0; i <= j; ++i) col[i] = hh[i * M + c] + hh[nd + i * M + c];
                const double hnext = std::sqrt(hn[c]);
                col[j + 1] = hnext;
                double *cc = cs.data() + c * R, *ss = sn.data() + c * R, *gc = g.data() + c * (R + 1);
                for (int i = 0; i < j; ++i) {
                    const double a = col[i], b = col[i + 1];
                    col[i] = cc[i] * a + ss[i] * b;
                    col[i + 1] = -ss[i] * a + cc[i] * b;
                }
                const double a = col[j], b = col[j + 1];
                const double rr = std::hypot(a, b);
                cc[j] = rr > 0.0 ? a / rr : 1.0;
                ss[j] = rr > 0.0 ? b / rr : 0.0;
                col[j] = rr;
                col[j + 1] = 0.0;
                gc[j + 1] = -ss[j] * gc[j];
                gc[j] = cc[j] * gc[j];
                const bool grow = hnext > 1e-300 * beta[c];
                if (std::fabs(gc[j + 1]) <= tgt[c] || !grow) {
                    live[c] = 0;  // this column stops here; its later vectors are zero
                } else {
                    sc[c] = 1.0 / hnext;
                    more = true;
                }
            }
            // the columns still running continue with V_{j+1} = W / hnext
            RMGE_TRY(hipMemcpyAsync(scl, sc.data(), sizeof(double) * M, hipMemcpyHostToDevice, s));
            RMGE_TRY(bscale(Vn, W, m, n, mi, scl, s));
            if (!more) break;
        }
        if (k == 0) break;
        // per column: R y = g over the steps it took, then X += Z y
        std::fill(hy.begin(), hy.end(), 0.0);
        for (size_t c = 0; c < M; ++c) {
            if (!active[c]) continue;
            // the steps this column took: up to where it stopped (its zero vectors after)
            int kc = 0;
            for (int i = 0; i < k; ++i)
                if (H[(c * R + i) * (R + 1) + i] != 0.0) kc = i + 1; else break;
            const double *gc = g.data() + c * (R + 1);
            std::vector<double> y(static_cast<size_t>(kc), 0.0);
            for (int i = kc - 1; i >= 0; --i) {
                double t = gc[i];
                for (int l = i + 1; l < kc; ++l) t -= H[(c * R + l) * (R + 1) + i] * y[l];
                const double d = H[(c * R + i) * (R + 1) + i];
                y[i] = d != 0.0 ? t / d : 0.0;
            }
            for (int i = 0; i < kc; ++i) hy[i * M + c] = y[i];
        }
        RMGE_TRY(hipMemcpyAsync(yv, hy.data(), sizeof(double) * k * M, hipMemcpyHostToDevice, s));
        RMGE_TRY(blincomb(X, ldx, Z, n, mi, k, yv, 1.0, s));
        // the Hessenberg columns of this cycle are rebuilt from zero next cycle
        std::fill(H.begin(), H.end(), 0.0);
    }
    rs = solve_sync_error(f);
    if (rs != RMGE_OK) return rs;
    double w0 = 0.0, w1 = 0.0;
    bool all_ok = true;
    for (size_t c = 0; c < M; ++c) {
        w0 = (eta0[c] > w0 || eta0[c] != eta0[c]) ? eta0[c] : w0;
        w1 = (eta[c] > w1 || eta[c] != eta[c]) ? eta[c] : w1;
        if (!(eta[c] <= tol)) all_ok = false;
    }
    loc.iters = total;
    loc.eta0 = w0;
    loc.eta = w1;
    loc.converged = all_ok ? 1 : 0;
    if (st) *st = loc;
    return all_ok ? RMGE_OK : RMGE_NOT_CONVERGED;
}

rmge_status check_factor_args(const double *A, int64_t n, int64_t lda, int32_t kind,
                              int32_t block, int32_t prec, int32_t pivot = RMGE_PIVOT_NONE) {
    if (!A || n < 1 || lda < n || n > (int64_t(1) << 20)) return RMGE_EINVAL;
    if (pivot != RMGE_PIVOT_NONE && pivot != RMGE_PIVOT_BLOCK) return RMGE_EINVAL;
    if (kind < RMGE_MULT_NONE || kind > RMGE_MULT_UNITARY_CIRCULANT) return RMGE_EINVAL;
    if (block < 0 || block > kMaxBlock) return RMGE_EINVAL;
    if (prec != RMGE_F64 && prec != RMGE_F32 && prec != RMGE_BF16 && prec != RMGE_F32_BF16X2)
        return RMGE_EINVAL;
    if (is_fft_kind(kind) && fft_period(kind, n) == 0)
        return RMGE_EINVAL;
    return RMGE_OK;
}

// ------------------------------------------------- no-allocation scratch
//
// rmge_precondition_noalloc keeps the multiplier's workspace in this fixed
// array instead of an allocation (for callers that cannot allocate: code under
// graph capture, serving loops).  In host code `scratch` is only a stand-in
// symbol: kernels receive the device address that hipGetSymbolAddress gives,
// looked up once per device (each GPU holds its own copy of the array).
constexpr int64_t kNoallocScratchDoubles = int64_t(1) << 20;  // 8 MiB
__device__ __align__(256) double scratch[kNoallocScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

rmge_status noalloc_scratch(double **out) {
    int dev = 0;
    RMGE_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return RMGE_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        RMGE_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return RMGE_EDEVICE;
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return RMGE_OK;
}

// Doubles of workspace rmge_precondition needs for (kind, n) with FFT period m:
// G for a dense Gaussian multiplier; parameters, period-m kernel, half
// spectrum and twiddles for the FFT kinds.
int64_t noalloc_doubles(int32_t kind, int64_t n, int m) {
    if (kind == RMGE_MULT_GAUSSIAN) return n * n;
    if (m) return 2 * n + m + 4 * (m / 2 + 1);
    return 0;
}

}  // namespace

extern "C" {

rmge_status rmge_factor_pivoted(const double *A, int64_t n, int64_t lda, int32_t kind,
                                uint64_t seed, int32_t block, int32_t prec, int32_t pivot,
                                void *hip_stream, rmge_factors **out) {
    if (!out) return RMGE_EINVAL;
    rmge_status rs = check_factor_args(A, n, lda, kind, block, prec, pivot);
    if (rs != RMGE_OK) return rs;
    if (!device_ok()) return RMGE_EDEVICE;
    rmge_factors *f = new (std::nothrow) rmge_factors();
    if (!f) return RMGE_ENOMEM;
    f->n = n;
    f->lda = lda;
    f->ld = round_up(n, 64);
    f->kind = kind;
    f->prec = (prec == RMGE_F32_BF16X2 || prec == RMGE_BF16) ? RMGE_F32 : prec;
    f->split16 = (prec == RMGE_F32_BF16X2 || prec == RMGE_BF16) && kind == RMGE_MULT_GAUSSIAN;
    f->upd_terms = prec == RMGE_F32_BF16X2 ? 3 : prec == RMGE_BF16 ? 1 : 0;
    f->block = block == 0 ? kMaxBlock : block;
    f->pivot = pivot;
    f->seed = seed;
    f->stream = static_cast<hipStream_t>(hip_stream);
    f->A = A;
    f->m = is_fft_kind(kind) ? fft_period(kind, n) : 0;
    rs = alloc_handle(f);
    if (rs != RMGE_OK) {
        free_handle(f);
        return rs;
    }
    rs = (f->prec == RMGE_F32) ? run_factor<float>(f) : run_factor<double>(f);
    if (rs == RMGE_OK || rs == RMGE_ZERO_PIVOT || rs == RMGE_NONFINITE) {
        *out = f;
        return rs;
    }
    free_handle(f);
    return rs;
}

rmge_status rmge_factor_ex(const double *A, int64_t n, int64_t lda, int32_t kind, uint64_t seed,
                           int32_t block, int32_t prec, void *hip_stream, rmge_factors **out) {
    return rmge_factor_pivoted(A, n, lda, kind, seed, block, prec, RMGE_PIVOT_NONE, hip_stream,
                               out);
}

rmge_status rmge_factor(const double *A, int64_t n, int32_t kind, uint64_t seed, int32_t block,
                        rmge_factors **out) {
    return rmge_factor_ex(A, n, n, kind, seed, block, RMGE_F64, nullptr, out);
}

rmge_status rmge_refactor(rmge_factors *f, const double *A, int64_t lda, uint64_t seed) {
    if (!f || !A || lda < f->n) return RMGE_EINVAL;
    f->A = A;
    f->lda = lda;
    f->seed = seed;
    return (f->prec == RMGE_F32) ? run_factor<float>(f) : run_factor<double>(f);
}

rmge_status rmge_solve(const rmge_factors *fc, const double *B, int64_t nrhs, int64_t ldb,
                       double *X, int64_t ldx, int32_t max_refine, double tol,
                       rmge_solve_stats *st) {
    rmge_factors *f = const_cast<rmge_factors *>(fc);
    if (!f || !B || !X || nrhs < 1 || ldb < nrhs || ldx < nrhs || max_refine < 0 ||
        max_refine > 16 || X == B)
        return RMGE_EINVAL;
    if (f->host_st.code == 4) return RMGE_ZERO_PIVOT;
    if (f->host_st.code == 5) return RMGE_NONFINITE;
    return (f->prec == RMGE_F32) ? run_solve<float>(f, B, nrhs, ldb, X, ldx, max_refine, tol, st)
                                 : run_solve<double>(f, B, nrhs, ldb, X, ldx, max_refine, tol, st);
}

rmge_status rmge_solve_gmres(const rmge_factors *fc, int32_t trans, const double *B, int64_t nrhs,
                             int64_t ldb, double *X, int64_t ldx, int32_t max_iters,
                             int32_t restart, double tol, rmge_solve_stats *st) {
    rmge_factors *f = const_cast<rmge_factors *>(fc);
    if (!f || !B || !X || nrhs < 1 || ldb < nrhs || ldx < nrhs || max_iters < 0 || X == B ||
        restart < 1 || restart > kMaxRestart || !(tol > 0.0) || (trans != 0 && trans != 1))
        return RMGE_EINVAL;
    if (f->host_st.code == 4) return RMGE_ZERO_PIVOT;
    if (f->host_st.code == 5) return RMGE_NONFINITE;
    if (nrhs > 1 && nrhs <= 64)
        return (f->prec == RMGE_F32)
                   ? run_gmres_block<float>(f, trans != 0, B, nrhs, ldb, X, ldx, max_iters,
                                            restart, tol, st)
                   : run_gmres_block<double>(f, trans != 0, B, nrhs, ldb, X, ldx, max_iters,
                                             restart, tol, st);
    return (f->prec == RMGE_F32)
               ? run_gmres<float>(f, trans != 0, B, nrhs, ldb, X, ldx, max_iters, restart, tol, st)
               : run_gmres<double>(f, trans != 0, B, nrhs, ldb, X, ldx, max_iters, restart, tol,
                                   st);
}

rmge_status rmge_solve_adjoint(const rmge_factors *fc, const double *W, int64_t nrhs,
                               int64_t ldw, double *Y, int64_t ldy) {
    rmge_factors *f = const_cast<rmge_factors *>(fc);
    if (!f || !W || !Y || nrhs < 1 || ldw < nrhs || ldy < nrhs) return RMGE_EINVAL;
    if (f->host_st.code == 4) return RMGE_ZERO_PIVOT;
    if (f->host_st.code == 5) return RMGE_NONFINITE;
    return (f->prec == RMGE_F32) ? run_adjoint<float>(f, W, nrhs, ldw, Y, ldy, 0, 0.0, nullptr)
                                 : run_adjoint<double>(f, W, nrhs, ldw, Y, ldy, 0, 0.0, nullptr);
}

rmge_status rmge_solve_adjoint_ex(const rmge_factors *fc, const double *W, int64_t nrhs,
                                  int64_t ldw, double *Y, int64_t ldy, int32_t max_refine,
                                  double tol, rmge_solve_stats *st) {
    rmge_factors *f = const_cast<rmge_factors *>(fc);
    if (!f || !W || !Y || nrhs < 1 || ldw < nrhs || ldy < nrhs || W == Y || max_refine < 0 ||
        max_refine > 16)
        return RMGE_EINVAL;
    if (f->host_st.code == 4) return RMGE_ZERO_PIVOT;
    if (f->host_st.code == 5) return RMGE_NONFINITE;
    rmge_solve_stats loc{};
    return (f->prec == RMGE_F32)
               ? run_adjoint<float>(f, W, nrhs, ldw, Y, ldy, max_refine, tol, st ? st : &loc)
               : run_adjoint<double>(f, W, nrhs, ldw, Y, ldy, max_refine, tol, st ? st : &loc);
}

rmge_status rmge_grad_A(const double *GB, int64_t ldgb, const double *X, int64_t ldx, int64_t n,
                        int64_t nrhs, double *GA, int64_t ldga, void *hip_stream) {
    if (!GB || !X || !GA || n < 1 || n > (int64_t(1) << 20) || nrhs < 1 || nrhs > 64 ||
        ldgb < nrhs || ldx < nrhs || ldga < n)
        return RMGE_EINVAL;
    if (!device_ok()) return RMGE_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    RMGE_TRY(grad_a(GB, ldgb, X, ldx, n, static_cast<int>(nrhs), GA, ldga, s));
    return from_hip(hipStreamSynchronize(s));
}

rmge_status rmge_factor_stats_get(const rmge_factors *fc, rmge_factor_stats *s) {
    rmge_factors *f = const_cast<rmge_factors *>(fc);
    if (!f || !s) return RMGE_EINVAL;
    if (!f->stats_done && f->host_st.code == 0) {
        hipError_t e = (f->prec == RMGE_F32)
                           ? lu_stats<float>(static_cast<const float *>(f->lu), f->ld, f->n,
                                             f->scal, f->stream)
                           : lu_stats<double>(static_cast<const double *>(f->lu), f->ld, f->n,
                                              f->scal, f->stream);
        if (e != hipSuccess) return from_hip(e);
        double h[3];
        RMGE_TRY(hipMemcpyAsync(h, f->scal, sizeof(h), hipMemcpyDeviceToHost, f->stream));
        RMGE_TRY(hipStreamSynchronize(f->stream));
        f->stats.min_abs_pivot = h[1];
        f->stats.growth = h[2] > 0.0 ? h[0] / h[2] : 0.0;
        f->stats_done = true;
    }
    *s = f->stats;
    return RMGE_OK;
}

rmge_status rmge_factor_times(const rmge_factors *f, double *ms3) {
    if (!f || !ms3) return RMGE_EINVAL;
    ms3[0] = f->stats.ms_multiplier;
    ms3[1] = f->stats.ms_product;
    ms3[2] = f->stats.ms_factor;
    return RMGE_OK;
}

rmge_status rmge_factor_update_time(const rmge_factors *f, double *ms, double *flops) {
    if (!f || !ms || !flops) return RMGE_EINVAL;
    *ms = f->ms_update;
    *flops = f->upd_flops;
    return RMGE_OK;
}

rmge_status rmge_factors_lu(const rmge_factors *f, double *LU, int64_t ld) {
    if (!f || !LU || ld < f->n) return RMGE_EINVAL;
    hipError_t e = (f->prec == RMGE_F32)
                       ? convert_2d<float, double>(static_cast<const float *>(f->lu), f->ld, LU,
                                                   ld, f->n, f->n, f->stream)
                       : convert_2d<double, double>(static_cast<const double *>(f->lu), f->ld, LU,
                                                    ld, f->n, f->n, f->stream);
    if (e != hipSuccess) return from_hip(e);
    return from_hip(hipStreamSynchronize(f->stream));
}

rmge_status rmge_factors_perm(const rmge_factors *f, int32_t *perm) {
    if (!f || !perm) return RMGE_EINVAL;
    if (f->pivot)
        RMGE_TRY(hipMemcpyAsync(perm, f->piv, sizeof(int) * static_cast<size_t>(f->n),
                                hipMemcpyDeviceToDevice, f->stream));
    else
        RMGE_TRY(iota(perm, f->n, f->stream));
    return from_hip(hipStreamSynchronize(f->stream));
}

int64_t rmge_param_count(int32_t kind, int64_t n) {
    if (n < 1) return 0;
    switch (kind) {
    case RMGE_MULT_GAUSSIAN: return n * n;
    case RMGE_MULT_CIRCULANT: return n;
    case RMGE_MULT_TOEPLITZ: return 2 * n - 1;
    case RMGE_MULT_UNITARY_CIRCULANT: return n;
    default: return 0;
    }
}

rmge_status rmge_multiplier_params(int32_t kind, int64_t n, uint64_t seed, double *out,
                                   void *hip_stream) {
    const int64_t cnt = rmge_param_count(kind, n);
    if (!out || cnt == 0) return RMGE_EINVAL;
    if (!device_ok()) return RMGE_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (kind == RMGE_MULT_UNITARY_CIRCULANT) {  // the first column, from n phases
        double *phi = nullptr;
        RMGE_TRY(hipMalloc(&phi, sizeof(double) * static_cast<size_t>(n)));
        hipError_t e = launch_uniforms_f64(phi, n, seed, static_cast<uint64_t>(kind), s);
        if (e == hipSuccess) e = unitary_column(phi, n, out, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        (void)hipFree(phi);
        return from_hip(e);
    }
    RMGE_TRY(launch_normals_f64(out, cnt, seed, static_cast<uint64_t>(kind), s));
    return from_hip(hipStreamSynchronize(s));
}

rmge_status rmge_precondition(const double *A, int64_t n, int64_t lda, int32_t kind,
                              uint64_t seed, double *M, int64_t ldm, void *hip_stream) {
    if (!M || ldm < n || M == A) return RMGE_EINVAL;
    rmge_status rs = check_factor_args(A, n, lda, kind, 0, RMGE_F64);
    if (rs != RMGE_OK) return rs;
    if (!device_ok()) return RMGE_EDEVICE;
    rmge_factors f;
    f.n = n;
    f.lda = lda;
    f.ld = ldm;
    f.kind = kind;
    f.seed = seed;
    f.stream = static_cast<hipStream_t>(hip_stream);
    f.A = A;
    f.lu = M;
    f.m = is_fft_kind(kind) ? fft_period(kind, n) : 0;
    hipError_t e = hipSuccess;
    if (kind == RMGE_MULT_GAUSSIAN) e = hipMalloc(&f.G, sizeof(double) * static_cast<size_t>(n * n));
    if (e == hipSuccess && f.m) {
        const int L = f.m / 2;
        e = hipMalloc(&f.params, sizeof(double) * static_cast<size_t>(2 * n));
        if (e == hipSuccess) e = hipMalloc(&f.hker, sizeof(double) * static_cast<size_t>(f.m));
        if (e == hipSuccess) e = hipMalloc(&f.hhat, sizeof(double) * 2 * static_cast<size_t>(L + 1));
        if (e == hipSuccess) e = hipMalloc(&f.tw, sizeof(double) * 2 * static_cast<size_t>(L + 1));
        if (e == hipSuccess) e = fft_twiddles(f.m, f.tw, f.stream);
    }
    if (e == hipSuccess) e = precondition<double>(&f);
    if (e == hipSuccess) e = hipStreamSynchronize(f.stream);
    void *tmp[] = {f.G, f.params, f.hker, f.hhat, f.tw};
    for (void *p : tmp)
        if (p) (void)hipFree(p);
    f.lu = nullptr;
    return from_hip(e);
}

rmge_status rmge_precondition_noalloc(const double *A, int64_t n, int64_t lda, int32_t kind,
                                      uint64_t seed, double *M, int64_t ldm, void *hip_stream) {
    if (!M || ldm < n || M == A) return RMGE_EINVAL;
    rmge_status rs = check_factor_args(A, n, lda, kind, 0, RMGE_F64);
    if (rs != RMGE_OK) return rs;
    const int m = is_fft_kind(kind) ? fft_period(kind, n) : 0;
    if (noalloc_doubles(kind, n, m) > kNoallocScratchDoubles) return RMGE_EINVAL;
    if (!device_ok()) return RMGE_EDEVICE;
    double *scr = nullptr;
    if ((rs = noalloc_scratch(&scr)) != RMGE_OK) return rs;
    rmge_factors f;
    f.n = n;
    f.lda = lda;
    f.ld = ldm;
    f.kind = kind;
    f.seed = seed;
    f.stream = static_cast<hipStream_t>(hip_stream);
    f.A = A;
    f.lu = M;
    f.m = m;
    if (kind == RMGE_MULT_GAUSSIAN) {
        f.G = scr;
    } else if (m) {  // the same carving as the handle's buffers, end to end
        const int L = m / 2;
        f.params = scr;
        f.hker = f.params + 2 * n;
        f.hhat = f.hker + m;
        f.tw = f.hhat + 2 * (L + 1);
    }
    hipError_t e = m ? fft_twiddles(m, f.tw, f.stream) : hipSuccess;
    if (e == hipSuccess) e = precondition<double>(&f);
    f.lu = nullptr;
    return from_hip(e);
}

rmge_status rmge_schur_update_f32(int64_t M, int64_t N, int64_t K, const float *D, int64_t ldd,
                                  const float *E, int64_t lde, float *C, int64_t ldc,
                                  int32_t terms, void *hip_stream) {
    if (!D || !E || !C || M < 0 || N < 0 || K < 0 || M > INT32_MAX || N > INT32_MAX ||
        K > kMaxBlock || ldd < K || lde < N || ldc < N || (terms != 0 && terms != 1 && terms != 3))
        return RMGE_EINVAL;
    if (M == 0 || N == 0 || K == 0) return RMGE_OK;
    if (!device_ok()) return RMGE_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (terms == 0) {
        RMGE_TRY(gemm_f32(kGemmUpdate, M, N, K, -1.0f, D, ldd, E, lde, 1.0f, C, ldc, nullptr, s));
        return from_hip(hipStreamSynchronize(s));
    }
    const int64_t rows = round_up(M > N ? M : N, 256), ldk = round_up(K, 32);
    if (2 * terms * 2 * rows * ldk > INT32_MAX) return RMGE_EINVAL;
    uint16_t *ws = nullptr;
    RMGE_TRY(hipMalloc(&ws, sizeof(uint16_t) * static_cast<size_t>(2 * terms * rows * ldk)));
    hipError_t e = update_bf16(terms, M, N, K, D, ldd, E, lde, C, ldc, ws, ldk, rows, nullptr, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(ws);
    return from_hip(e);
}

void rmge_destroy(rmge_factors *f) { free_handle(f); }

const char *rmge_status_string(int32_t s) {
    switch (s) {
    case RMGE_OK: return "ok";
    case RMGE_EINVAL: return "invalid argument";
    case RMGE_ENOMEM: return "device allocation failed";
    case RMGE_EDEVICE: return "HIP runtime error or no gfx950 device";
    case RMGE_ZERO_PIVOT: return "zero pivot: the preprocessed matrix is not strongly nonsingular";
    case RMGE_NONFINITE: return "non-finite pivot";
    case RMGE_NOT_CONVERGED: return "refinement did not reach the tolerance";
    default: return "unknown status";
    }
}

int32_t rmge_version(void) { return 100; }

}  // extern "C"
