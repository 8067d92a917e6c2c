// Internal declarations of the gfx950 library: device status word, launchers.
// Every launcher enqueues on the given stream and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rmge {

// Device-resident status of a factorization.  `code` is 0 while every pivot
// seen so far is finite and nonzero; the first kernel that meets a zero or
// non-finite pivot stores its global index in `info` and sets `code`
// (4 = zero pivot, 5 = non-finite).  Later kernels read `code` and exit early.
struct DevStatus {
    long long info;
    int code;
    int pad;
};

// p[i] when `in` holds, else 0.  The load is issued unconditionally (from
// p[0], which must be readable, when `in` is false): a load under a branch
// makes the wave wait for it where the branch rejoins, so a run of guarded
// loads would be serialised one memory latency at a time.
template <typename T>
__device__ inline T load_if(const T *p, int64_t i, bool in) {
    const T x = p[in ? i : 0];
    return in ? x : T(0);
}

constexpr int kLeaf = 128;      // largest diagonal block factored in LDS
constexpr int kMaxBlock = 256;  // largest panel width

// ---------------------------------------------------------------- rng.hip
hipError_t launch_normals_f64(double *out, int64_t count, uint64_t seed, uint64_t stream,
                              hipStream_t s);
hipError_t launch_normals_f32(float *out, int64_t count, uint64_t seed, uint64_t stream,
                              hipStream_t s);
// The multiplier parameters of many systems in one launch: system s draws
// cnt[s] normals of stream stream[s] (1: FP32 into g32 + off[s]; otherwise FP64
// into g64 + off[s]) with seed[s]; chunk_start: count + 1 prefix sums of
// ceil(cnt / 1024).  All arrays on the device.
hipError_t batch_normals(int count, int total_chunks, const int *chunk_start, const int64_t *cnt,
                         const int *stream, const uint64_t *seed, const int64_t *off, float *g32,
                         double *g64, hipStream_t s);
// count uniforms in (0, 1) of the same generator (element e = u_{e mod 4} of block e / 4).
hipError_t launch_uniforms_f64(double *out, int64_t count, uint64_t seed, uint64_t stream,
                               hipStream_t s);

// --------------------------------------------------------------- gemm.hip
// C = alpha * A * B + beta * C, row-major.  A is M x K (lda), B is K x N (ldb),
// C is M x N (ldc); C must not overlap A or B.  `shape` picks the tiling:
// kGemmProduct for large K (M = A H), kGemmUpdate for the Schur-complement
// update (K = panel width).  `abort` (device int, may be null): if nonzero at
// kernel start, do nothing.  `absmax` (device double, may be null): maxed
// atomically with max |C| of the written results.
enum GemmShape { kGemmProduct = 0, kGemmUpdate = 1 };
hipError_t gemm_f64(int shape, int64_t M, int64_t N, int64_t K, double alpha, const double *A,
                    int64_t lda, const double *B, int64_t ldb, double beta, double *C, int64_t ldc,
                    const int *abort, hipStream_t s, double *absmax = nullptr);
hipError_t gemm_f32(int shape, int64_t M, int64_t N, int64_t K, float alpha, const float *A,
                    int64_t lda, const float *B, int64_t ldb, float beta, float *C, int64_t ldc,
                    const int *abort, hipStream_t s, double *absmax = nullptr);
// FP32 product whose A operand is stored in FP64 (rounded to FP32 on load).
// The split-BF16 product C (M x N FP32) = (A_h + A_l) Ht^T on BF16 matrix cores:
// A_h, A_l (>= round_up(M, 256) rows x lda) and Ht (>= round_up(N, 256) rows x
// ldh) BF16 bit patterns, zero-padded; Kp % 32 == 0, lda, ldh % 8 == 0.
hipError_t gemm_bf16x2(int64_t M, int64_t N, int64_t Kp, const uint16_t *Ah, const uint16_t *Al,
                       int64_t lda, const uint16_t *Ht, int64_t ldh, float *C, int64_t ldc,
                       hipStream_t s, double *absmax);
// A (FP64) -> A_h = bf16(A), A_l = bf16(A - A_h); H (FP32, n x n) rounded to
// BF16 in place and transposed into Ht.
hipError_t split_bf16(const double *A, int64_t lda, int64_t n, uint16_t *ah, uint16_t *al,
                      int64_t ldk, hipStream_t s);
hipError_t round_h_bf16(float *H, int64_t n, uint16_t *Ht, int64_t ldk, hipStream_t s);
// The same H as launch_normals_f32 followed by round_h_bf16, in one pass:
// G (n x n FP32, BF16-rounded values) and Ht (transposed BF16 bits, pitch
// ldk >= round_up(n, 64), ldk % 8 == 0); needs n % 4 == 0.
hipError_t normals_bf16t(float *G, uint16_t *Ht, int64_t n, int64_t ldk, uint64_t seed,
                         uint64_t stream, hipStream_t s);
// Schur update C <- C - D E (D: M x K, E: K x N, C: M x N, all FP32 row-major)
// on the BF16 matrix cores with FP32 accumulation.  terms = 3: each operand
// cut into three BF16 terms and the six leading cross products formed (the
// FP32 product's accuracy); terms = 1: each operand rounded once to BF16.
// ws: workspace of 2 * terms * rows * ldk BF16 values, rows % 256 == 0 and
// >= round_up(max(M, N), 256), ldk % 8 == 0 and >= round_up(K, 32); its
// contents on entry do not matter.
hipError_t update_bf16(int terms, int64_t M, int64_t N, int64_t K, const float *D, int64_t ldd,
                       const float *E, int64_t lde, float *C, int64_t ldc, uint16_t *ws,
                       int64_t ldk, int64_t rows, const int *abort, hipStream_t s);
// Batched M_s = A_s G_s (FP64 A rounded to FP32, FP32 G and M, square n_s x n_s,
// ld = n_s) over `count` systems; tile_start (count + 1 ints, device): prefix
// sums of ceil(n_s / 64)^2; nsys, a_off, g_off, m_off: device arrays.
hipError_t batch_gemm_f32(int count, int total_tiles, const int *tile_start, const int *nsys,
                          const int64_t *a_off, const int64_t *g_off, const int64_t *m_off,
                          const double *A, const float *G, float *M, hipStream_t s);
// The same in FP64 (G's FP32 values as doubles, M FP64) for the systems whose
// flag[sys[s]] is nonzero (sys, flag: device arrays; sys maps the list to the
// caller's system index).
hipError_t batch_gemm_f64(int count, int total_tiles, const int *tile_start, const int *nsys,
                          const int *sys, const int *flag, const int64_t *a_off,
                          const int64_t *g_off, const int64_t *m_off, const double *A,
                          const float *G, double *M, hipStream_t s);
// Y = beta Y + alpha M X on the FP64 matrix cores for 1 <= nrhs <= 16 right-hand
// sides (M: rows x cols of TM = double or float, X: cols x nrhs FP64, ld ldx).
template <typename TM>
hipError_t gemm_skinny(int64_t rows, int64_t cols, double alpha, const TM *Mat, int64_t ldm,
                       const double *X, int64_t ldx, double beta, double *Y, int64_t ldy,
                       int nrhs, hipStream_t s);
hipError_t gemm_f32_a64(int shape, int64_t M, int64_t N, int64_t K, float alpha, const double *A,
                        int64_t lda, const float *B, int64_t ldb, float beta, float *C,
                        int64_t ldc, const int *abort, hipStream_t s, double *absmax = nullptr);

// ----------------------------------------------------------------- lu.hip
// Factor the b x b diagonal block at `a` (b <= kLeaf) in place and write the
// inverses of the 32 x 32 diagonal sub-blocks of its unit-lower and upper
// factors into Linv and Uinv (compact: row 32 q + i holds row i of sub-block
// q's inverse, 32 columns).
// k0 = global index of the block's first pivot (the block sits at rows and
// columns k0 ..).  piv == nullptr: GENP.  Otherwise partial pivoting inside
// the block: rows are stored in pivot order and piv[k0 + t] receives the
// global row index that now sits at k0 + t.
template <typename T>
hipError_t leaf_lu(T *a, int64_t lda, int b, T *Linv, T *Uinv, int64_t k0, DevStatus *st, int *piv,
                   hipStream_t s);
// Inverses of all aligned 32 x 32 diagonal sub-blocks of the n x n packed
// factors at `a` (compact: row 32 q + i of Linv / Uinv holds row i of
// sub-block q's inverse); skipped if the factorization broke down.
template <typename T>
hipError_t diag_inverses(const T *a, int64_t lda, int64_t n, T *Linv, T *Uinv, const DevStatus *st,
                         hipStream_t s);
// In-place triangular solves with the factored pivot block at `lu` (width
// b <= kMaxBlock), by blocked substitution with the compact 32 x 32 diagonal
// inverses Linv / Uinv, both in one launch:
//   Cl (b x countl, ldcl) <- L^{-1} P Cl   (row t of P Cl is row rowsrc[t] -
//                                          rowbase of Cl, or row t when rowsrc is null)
//   Cr (countr x b, ldcr) <- Cr U^{-1}
// The two blocks must not overlap; abort must not be null.
template <typename T>
hipError_t trsm_pair(const T *lu, int64_t ld, int b, T *Cl, int64_t ldcl, int64_t countl,
                     const T *Linv, const int *rowsrc, int64_t rowbase, T *Cr, int64_t ldcr,
                     int64_t countr, const T *Uinv, const int *abort, hipStream_t s);
// After a pivoted factorization with panels of nb: apply every diagonal
// block's row exchanges (piv) to the multipliers left of its panel.
template <typename T>
hipError_t permute_left(T *a, int64_t ld, int64_t n, int nb, const int *piv, const int *abort,
                        hipStream_t s);
// Rows s0 .. s0 + w - 1 (w <= kLeaf) of columns cb .. ce - 1 take the values of
// rows piv[s0 + t] (one diagonal block's exchanges inside its own panel).
template <typename T>
hipError_t permute_rows(T *a, int64_t ld, int64_t s0, int w, int64_t cb, int64_t ce,
                        const int *piv, const int *abort, hipStream_t s);
// p[i] = i, i < n.
hipError_t iota(int *p, int64_t n, hipStream_t s);
// dst row (scatter ? scatter[i] : i) <- src row (gather ? gather[i] : i), i < rows.
template <typename T, typename U>
hipError_t convert_2d(const T *src, int64_t lds, U *dst, int64_t ldd, int64_t rows, int64_t cols,
                      hipStream_t s, const int *gather = nullptr, const int *scatter = nullptr);
// out3[0] = max |U|, out3[1] = min |u_kk| (preset to 0, +Inf); atomics.
template <typename T>
hipError_t lu_stats(const T *lu, int64_t ld, int64_t n, double *out3, hipStream_t s);
// out3[2] = max |M| over the n x n matrix (preset to 0); atomics.
template <typename T>
hipError_t abs_max(const T *m, int64_t ld, int64_t n, double *out3, hipStream_t s);

// -------------------------------------------------------------- solve.hip
// A whole triangular solve T X = B with the packed factors LU (ld) in one
// launch:
//   mode 0: L y = b (unit lower, forward)      mode 1: U y = b (upper, backward)
//   mode 2: U^T y = b (lower, forward)         mode 3: L^T y = b (unit upper, backward)
// Blocks of 64 rows are taken in dependency order by a ticket counter.
// Dinv: compact inverses of the aligned 32 x 32 diagonal sub-blocks of L
// (modes 0, 3) or U (modes 1, 2), from diag_inverses, with at least
// round_up(n, 64) rows.  X and B are FP64, n x ldx (nr <= 16 columns used; X
// may not alias B); the arithmetic is FP64 whatever the factors' type.  sync:
// device ints, [0] ticket counter, [1] error word (set to 1 if a wait timed
// out; the caller clears it).
template <typename T>
hipError_t trsv_full(int mode, const T *LU, int64_t ld, int64_t n, const T *Dinv, const double *B,
                     double *X, int64_t ldx, int nr, int *sync, hipStream_t s);
// FP64 inverses D_I of the 128 x 128 diagonal blocks of the packed factors
// (unit lower L, upper U), and W_I = D_I C_I with C_I the coupling of block I
// with its predecessor in the solve (L: block column I - 1; U: I + 1): row
// I0 + i of each output holds row i of block I's matrix; all four hold
// round_up(n, 128) rows of 128 doubles.
template <typename T>
hipError_t block_inverses128(const T *lu, int64_t ld, int64_t n, double *Linv, double *Uinv,
                             double *Wl, double *Wu, hipStream_t s);
// One right-hand side: mode 0 L y = b, mode 1 U y = b, in 128-row blocks with
// the block matrices above (Linv, Wl for mode 0; Uinv, Wu for mode 1).  B != X.
template <typename T>
hipError_t trsv128(int mode, const T *LU, int64_t ld, int64_t n, const double *Dinv,
                   const double *W, const double *B, double *X, int64_t ldx, int *sync,
                   hipStream_t s);
// Krylov helpers; basis vectors V_j stored contiguously (V + j * n), j < k <= 64.
// h[j] = V_j . w (+ h[j] if accumulate), deterministic; part: >= 256 * k doubles.
hipError_t mdot(const double *V, int64_t n, int k, const double *w, double *part, double *h,
                bool accumulate, hipStream_t s);
// w[i * ldw] += sign * sum_j V_j[i] h[j]  (h on the device).
hipError_t lincomb(double *w, int64_t ldw, const double *V, int64_t n, int k, const double *h,
                   double sign, hipStream_t s);
// dst[i] = alpha * src[i * lds].
// Block Krylov helpers for m <= 64 right-hand sides at once: basis block j is
// the n x m row-major matrix V + j n m.  bdot: h[j m + c] = V_j[:, c] . W[:, c]
// for j < k (part: >= 256 k m doubles; deterministic); blincomb:
// W[:, c] += sign sum_j h[j m + c] V_j[:, c]; bscale: dst = src diag(scale).
hipError_t bdot(const double *V, int64_t n, int m, int k, const double *W, int64_t ldw,
                double *part, double *h, bool accumulate, hipStream_t s);
hipError_t blincomb(double *W, int64_t ldw, const double *V, int64_t n, int m, int k,
                    const double *h, double sign, hipStream_t s);
hipError_t bscale(double *dst, const double *src, int64_t lds, int64_t n, int m,
                  const double *scale, hipStream_t s);
hipError_t scale_copy(double *dst, const double *src, int64_t lds, int64_t n, double alpha,
                      hipStream_t s);
// y = beta * y + alpha * M x  (rows of M; FP64 accumulation).  M: rows x cols (ldm),
// x: cols x nrhs (ldx), y: rows x nrhs (ldy).  rowmax (nrhs <= 4 only): also
// max(*rowmax, ||M||_inf) into *rowmax, from the same reads of M.
template <typename TM, typename TX, typename TY>
hipError_t gemv_n(int64_t rows, int64_t cols, double alpha, const TM *Mat, int64_t ldm,
                  const TX *x, int64_t ldx, double beta, TY *y, int64_t ldy, int nrhs,
                  hipStream_t s, double *rowmax = nullptr);
// y = M^T x (two passes, deterministic).  work: >= ceil(rows/256) * cols * nrhs doubles.
template <typename TM, typename TX, typename TY>
hipError_t gemv_t(int64_t rows, int64_t cols, const TM *Mat, int64_t ldm, const TX *x,
                  int64_t ldx, TY *y, int64_t ldy, int nrhs, double *work, hipStream_t s);
// norms[0..nrhs) = max_i |v[i][r]| for v = n x nrhs (ld), atomically maxed into norms.
hipError_t colmax_abs(const double *v, int64_t ld, int64_t n, int nrhs, double *norms,
                      hipStream_t s);
// out[0] = max_i sum_j |A[i][j]|.
hipError_t norm_inf(const double *A, int64_t lda, int64_t n, double *out, hipStream_t s);
// x = beta x + d (both n x nrhs, own leading dimensions); with `scatter`, row i of d
// goes to row scatter[i] of x.
template <typename TS>
hipError_t axpby_2d(const TS *d, int64_t ldd, double *x, int64_t ldx, int64_t n, int nrhs,
                    double beta, hipStream_t s, const int *scatter = nullptr);
// out[0] = max(out[0], ||A||_1) (max column sum of |A|; out preset to 0).
// work: >= ceil(n / 256) * n doubles.
hipError_t norm_one(const double *A, int64_t lda, int64_t n, double *work, double *out,
                    hipStream_t s);
hipError_t fill_f64(double *p, int64_t count, double value, hipStream_t s);
// y = beta y + H x (one right-hand side, FP64 accumulation; x, y strided by
// ldx, ldy) with H given transposed as BF16 bits: Ht (>= n rows x ldk, ldk % 8
// == 0 and >= round_up(n, 8), zero in columns [n, ldk)).  part: >=
// gemv_ht_blocks(n) * n doubles of scratch.
int64_t gemv_ht_blocks(int64_t n);
hipError_t gemv_ht(int64_t n, const uint16_t *Ht, int64_t ldk, const double *x, int64_t ldx,
                   double beta, double *y, int64_t ldy, double *part, hipStream_t s);
// GA = -GB X^T (n x n, ldga; GB, X: n x nrhs with their leading dimensions; nrhs <= 64,
// n <= 2^20).
hipError_t grad_a(const double *GB, int64_t ldgb, const double *X, int64_t ldx, int64_t n,
                  int nrhs, double *GA, int64_t ldga, hipStream_t s);

// ---------------------------------------------------------------- fft.hip
// Real FFT correlation / convolution of vectors with a fixed real kernel h of
// period m (a power of two, 2 <= m <= 16384), through a complex FFT of length
// L = m/2 staged in LDS.
//   tw:       twiddle table e^{-i pi j / L}, j = 0..L (complex, built by fft_twiddles).
//   hhat:     half spectrum hhat[f] = sum_d h[d] e^{-2 pi i f d / m}, f = 0..L.
//   vectors:  for each of `count` inputs x (length n <= m, zero padded),
//             y_j = sum_k x_k h[(k - j) mod m]   (correlate, conj = 1)
//             y_j = sum_k h[(j - k) mod m] x_k   (convolve,  conj = 0)
//             for j < n, written as out = beta * out + y.
//   Vector v, element k lives at in[v * vstride_in + k * estride_in].
hipError_t fft_twiddles(int m, double *tw, hipStream_t s);
// First column c (n values) of the random real unitary circulant from the
// phases phi (n uniforms; those past n/2 unused): the spectrum is
// u_j = e^{2 pi i phi_j}, u_{n-j} = conj(u_j) for 0 < j < n/2, u_0 and (even n)
// u_{n/2} = +1 if their phase is below 1/2 else -1; c = Omega^{-1} u,
// c_k = (1/n) sum_j u_j e^{-2 pi i j k / n}.
hipError_t unitary_column(const double *phi, int64_t n, double *c, hipStream_t s);
// The unitary circulant's half spectrum (m = n, a power of two, 2 <= n <= 16384)
// in closed form from its n phases: n/2 + 1 complex values into hhat.
hipError_t unitary_spectrum(const double *phi, int64_t n, double *hhat, hipStream_t s);
hipError_t fft_embed(int kind, const double *params, int64_t n, int m, double *h, hipStream_t s);
// Circulant multipliers of a batch (orders n_s <= 1024, periods m_s = 2^(logl_s + 1)
// <= 2048): per system, the period-m kernel h (h_pool + h_off[s]) from the first
// column (c_pool + c_off[s]) and its half spectrum (hh_pool + 2 hh_off[s] doubles,
// L_s + 1 complex); twiddles of period 2^(l + 1) at tw_pool + 2 tw_off[l].
hipError_t batch_fft_spectra(int count, const int *nsys, const int *logl, const int64_t *c_off,
                             const int64_t *h_off, const int64_t *hh_off, const int64_t *tw_off,
                             const double *c_pool, double *h_pool, double *hh_pool,
                             const double *tw_pool, hipStream_t s);
// Rows of M_s = A_s C_s (A FP64 at a_off[s], M of type TO (float or double) at
// m_off[s], ld = n_s) for all circulant systems; row_start: count + 1 prefix
// sums of n_s.  With flag != null, only the systems whose flag[sys[s]] is
// nonzero (sys, flag: device arrays).
template <typename TO>
hipError_t batch_fft_rows(int count, int total_rows, const int *row_start, const int *nsys,
                          const int *sys, const int *flag, const int *logl, const int64_t *a_off,
                          const int64_t *m_off, const int64_t *hh_off, const int64_t *tw_off,
                          const double *A, const double *hh_pool, const double *tw_pool, TO *M,
                          hipStream_t s);
hipError_t fft_spectrum(const double *h, int m, const double *tw, double *hhat, hipStream_t s);
template <typename TI, typename TO>
hipError_t fft_rows(const TI *in, int64_t vstride_in, int64_t estride_in, int64_t count,
                    int64_t n, int m, const double *tw, const double *hhat, int conj, double beta,
                    TO *out, int64_t vstride_out, int64_t estride_out, hipStream_t s,
                    double *absmax = nullptr);

}  // namespace rmge
