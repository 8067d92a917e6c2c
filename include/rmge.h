/*
 * rmge.h -- random-multiplier Gaussian elimination on AMD Instinct MI355X (gfx950).
 *
 * Solves A x = b for a nonsingular n x n matrix A by the method of Pan, Qian
 * and Yan, "Random multipliers numerically stabilize Gaussian and block
 * Gaussian elimination" (arXiv:1406.5802):
 *
 *   1. draw a random multiplier H (Definition defrndm: a standard Gaussian
 *      matrix; or a circulant matrix with a Gaussian first column, Section 6;
 *      or a Toeplitz matrix, the leading block of a larger random circulant);
 *   2. form M = A H (post-multiplication, Fact faprepr);
 *   3. factor M = L U by block Gaussian elimination with no pivoting
 *      (Section 3, eq. eqgenp applied to pivot blocks of `block` columns;
 *      in exact arithmetic the result does not depend on the block size,
 *      by the order-independence argument after eq. eqgenpin); or, as a
 *      variant, stop that recursion at small diagonal blocks and factor each
 *      with partial pivoting confined to the block (the black-box treatment
 *      of small pivot blocks that Section 3 allows): P M = L U with P a
 *      block-diagonal permutation;
 *   4. solve L U y = b and return x = H y (Fact faprepr), optionally followed
 *      by FP64 iterative refinement (Section 8.1 protocol).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All matrix and vector pointers are DEVICE pointers on the current HIP
 *   device, row-major, with the given leading dimension (in elements).
 *   Right-hand sides B and solutions X are n x nrhs, row-major.
 * - `hip_stream` is a hipStream_t passed as void*; NULL means the legacy
 *   default stream.  All work is enqueued on that stream.  Calls that return a
 *   numerical status (factor, solve) synchronise that stream before returning.
 * - Ownership: the caller owns A, B, X, W, Y.  The handle owns the factors,
 *   the multiplier state and its workspace.  The handle BORROWS A: A must stay
 *   alive and unchanged until rmge_destroy (it is read by refinement).
 *   A itself is never written.
 * - Errors are returned as rmge_status; nothing is thrown across the ABI.
 *   Device or allocation failures leave *out untouched (NULL-initialised by
 *   the caller is recommended).  On RMGE_ZERO_PIVOT / RMGE_NONFINITE the handle
 *   IS returned, with stats.info set; solves on such a handle return the same
 *   status without computing.
 * - Threads: handles are independent; calls on one handle must not overlap.
 */
#ifndef RMGE_H
#define RMGE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Multiplier kinds (the right multiplier H; post-multiplication only, the
 * case the paper proves, Section 4 after Fact faprepr). */
typedef enum {
    RMGE_MULT_NONE = 0,      /* H = I: plain GENP, shows breakdown (Corollary corec) */
    RMGE_MULT_GAUSSIAN = 1,  /* n x n i.i.d. N(0,1) (Definition defrndm), dense product */
    RMGE_MULT_CIRCULANT = 2, /* H[i][j] = c[(i-j) mod n], c i.i.d. N(0,1) (Section 6), FFT */
    RMGE_MULT_TOEPLITZ = 3   /* H[i][j] = t_{i-j}, 2n-1 i.i.d. N(0,1) parameters, FFT */
} rmge_mult;

/* Precision of the factors L, U (and of the multiplier product M = A H).
 * Residuals and solution updates of refinement are always FP64. */
typedef enum {
    RMGE_F64 = 0,       /* FP64 MFMA */
    RMGE_F32 = 1,       /* FP32 MFMA with FP32 accumulation; refine in FP64 */
    RMGE_F32_BF16X2 = 3 /* as RMGE_F32, but with a GAUSSIAN multiplier the product
                           M = A H runs on the BF16 matrix cores: H is drawn, then
                           rounded to BF16 (that rounded H is the multiplier, used
                           by the solves too), and A is split into two BF16 terms,
                           A = A_h + A_l + O(2^-18 |A|); M = A_h H + A_l H with FP32
                           accumulation.  The factors are FP32 as for RMGE_F32;
                           the Schur updates of trailing blocks of 2048 rows and
                           more also run on the BF16 matrix cores, each FP32
                           operand cut into three BF16 terms and the six leading
                           cross products formed (the dropped terms total at most
                           (2^-24 + 2^-34) of the product, one unit of FP32
                           rounding: the accuracy of an FP32 product).
                           Other multiplier kinds behave as RMGE_F32. */
} rmge_prec;

/* Row exchanges (rmge_factor_pivoted). */
typedef enum {
    RMGE_PIVOT_NONE = 0, /* GENP: no row exchanges (the paper's method) */
    /* Partial pivoting inside each diagonal block where the recursion stops.
     * The blocks: panels of `block` columns (the last may be narrower); a
     * panel wider than 128 is cut into its first 128 columns and the rest.
     * For column k the pivot is the entry of largest magnitude among the rows
     * of k's block at or below k (ties: the smaller original row index).
     * Rows never leave their block, so only the leading blocks at block
     * boundaries must be nonsingular (Theorem thnorms with those blocks). */
    RMGE_PIVOT_BLOCK = 1
} rmge_pivot;

typedef enum {
    RMGE_OK = 0,
    RMGE_EINVAL = 1,        /* bad argument (size, leading dimension, kind, block) */
    RMGE_ENOMEM = 2,        /* device allocation failed */
    RMGE_EDEVICE = 3,       /* HIP runtime error, or no gfx950 device */
    RMGE_ZERO_PIVOT = 4,    /* a pivot is exactly 0: M is not strongly nonsingular */
    RMGE_NONFINITE = 5,     /* a pivot is Inf or NaN */
    RMGE_NOT_CONVERGED = 6  /* refinement stopped above tol; X holds the last iterate */
} rmge_status;

typedef struct rmge_factors rmge_factors; /* opaque; owned by the library */

typedef struct {
    int64_t info;          /* 0-based index of the first zero / non-finite pivot, -1 if none */
    int32_t status;        /* RMGE_OK, RMGE_ZERO_PIVOT or RMGE_NONFINITE */
    int32_t block;         /* panel width used */
    double min_abs_pivot;  /* min_k |u_kk| (computed on demand, see rmge_factor_stats_get) */
    double growth;         /* max |U| / max |M| */
    double ms_multiplier;  /* device time of the last factorization: drawing H (and, for
                              FP32 factors with a Gaussian H, rounding A to FP32 once) */
    double ms_product;     /* device time: M = A H (one GEMM launch, or the FFT pass) */
    double ms_factor;      /* device time: the elimination (all pivot steps) */
} rmge_factor_stats;

typedef struct {
    int32_t iters;     /* refinement steps performed */
    int32_t converged; /* 1 if eta <= tol (or tol <= 0) */
    double eta0;       /* backward error before refinement */
    double eta;        /* final eta = max_r ||b_r - A x_r||_inf / (||A||_inf ||x_r||_inf + ||b_r||_inf) */
    double eta_hist[17]; /* eta after 0, 1, ... refinement steps (first iters + 1 entries) */
} rmge_solve_stats;

/* Factor A H = L U with the defaults: FP64, lda = n, default stream.
 * A: device, n x n row-major.  kind: rmge_mult.  seed: the multiplier's
 * random-number seed.  block: panel width, 1..256 (0 selects 256; 1 is
 * column-by-column GENP).  On success *out receives a new handle. */
rmge_status rmge_factor(const double *A, int64_t n, int32_t kind, uint64_t seed, int32_t block,
                        rmge_factors **out);

/* As rmge_factor with a leading dimension lda >= n, a factor precision
 * (rmge_prec) and a stream. */
rmge_status rmge_factor_ex(const double *A, int64_t n, int64_t lda, int32_t kind, uint64_t seed,
                           int32_t block, int32_t prec, void *hip_stream, rmge_factors **out);

/* As rmge_factor_ex with a choice of row exchanges (rmge_pivot).  With
 * RMGE_PIVOT_BLOCK the handle holds P M = L U; solves apply P, the adjoint
 * P^T, and rmge_factors_lu returns the rows in pivoted order.  A zero pivot
 * (all candidates of a column inside its block exactly 0) means the leading
 * block at that block boundary is singular; stats.info is its index. */
rmge_status rmge_factor_pivoted(const double *A, int64_t n, int64_t lda, int32_t kind,
                                uint64_t seed, int32_t block, int32_t prec, int32_t pivot,
                                void *hip_stream, rmge_factors **out);

/* Re-run the factorization of an existing handle on a new A of the same size
 * (same kind, precision, block and stream), reusing every allocation.  The new
 * A replaces the borrowed one. */
rmge_status rmge_refactor(rmge_factors *f, const double *A, int64_t lda, uint64_t seed);

/* X = A^{-1} B through A H Y = B, X = H Y (Fact faprepr), then refinement:
 * while step < max_refine and (tol <= 0 or eta > tol):
 *     R = B - A X (FP64);  D = H U^{-1} L^{-1} R (factor precision);  X += D (FP64).
 * tol <= 0 runs exactly max_refine steps (the paper's protocol: one).
 * B, X: device, n x nrhs, row-major, ldb, ldx >= nrhs; X may not alias B.
 * max_refine <= 16.  st may be NULL.  Returns RMGE_NOT_CONVERGED if tol > 0
 * and eta > tol after max_refine steps. */
rmge_status rmge_solve(const rmge_factors *f, const double *B, int64_t nrhs, int64_t ldb,
                       double *X, int64_t ldx, int32_t max_refine, double tol,
                       rmge_solve_stats *st);

/* X = A^{-1} B, refined by restarted flexible GMRES preconditioned by the
 * factors (GMRES-based iterative refinement; the paper's Section 8.1 uses
 * classical refinement, which stops contracting once the factors' backward
 * error times kappa(A H) nears 1, as FP32 factors of A G do at large n).
 * Per right-hand side: x0 = H U^{-1} L^{-1} P b; then outer steps
 * r = b - A x (FP64), inner iterations z_j = H U^{-1} L^{-1} P v_j (factor
 * precision), w = A z_j, FP64 Krylov basis orthogonalised twice, until the
 * least-squares residual estimate drops below tol (||A||_inf ||x||_inf +
 * ||b||_inf) / 2 or `restart` vectors are used; x += Z y.  Stops when
 * eta <= tol or after max_iters inner iterations for that right-hand side.
 * trans = 1 solves the adjoint system A^T x = b the same way (operator A^T,
 * preconditioner P^T L^{-T} U^{-T} H^T, eta with ||A||_1).
 * restart: 1..64.  tol > 0.  st->iters counts inner iterations over all
 * right-hand sides;
 * st->eta_hist holds eta at each outer check (first 17).  Returns
 * RMGE_NOT_CONVERGED if some right-hand side ends above tol.  Workspace:
 * (2 restart + 2) n doubles, kept by the handle. */
rmge_status rmge_solve_gmres(const rmge_factors *f, int32_t trans, const double *B, int64_t nrhs,
                             int64_t ldb, double *X, int64_t ldx, int32_t max_iters,
                             int32_t restart, double tol, rmge_solve_stats *st);

/* Y = A^{-T} W = L^{-T} U^{-T} H^T W (the adjoint, from A^{-1} = H (A H)^{-1},
 * Fact faprepr; P^T L^{-T} U^{-T} H^T W when pivoted).  Reuses L and U.
 * W, Y: device, n x nrhs, row-major. */
rmge_status rmge_solve_adjoint(const rmge_factors *f, const double *W, int64_t nrhs, int64_t ldw,
                               double *Y, int64_t ldy);

/* The adjoint with FP64 refinement: Y = A^{-T} W as above, then while
 * step < max_refine and (tol <= 0 or eta > tol):
 *     R = W - A^T Y (FP64);  Y += P^T L^{-T} U^{-T} H^T R,
 * with eta = max_r ||R_r||_inf / (||A||_1 ||Y_r||_inf + ||W_r||_inf) (the normwise
 * backward error of A^T y = w).  For FP32 factors the plain adjoint carries the
 * factors' accuracy only; this is how it reaches FP64 accuracy.  W, Y: device,
 * n x nrhs, Y may not alias W, max_refine <= 16, st may be NULL.  Returns
 * RMGE_NOT_CONVERGED if tol > 0 and eta > tol after max_refine steps. */
rmge_status rmge_solve_adjoint_ex(const rmge_factors *f, const double *W, int64_t nrhs,
                                  int64_t ldw, double *Y, int64_t ldy, int32_t max_refine,
                                  double tol, rmge_solve_stats *st);

/* Gradient with respect to A of a loss L(X) with X = A^{-1} B: given
 * GB = A^{-T} dL/dX (= dL/dB, from rmge_solve_adjoint), dL/dA = -GB X^T
 * (differentiating A X = B; the multiplier cancels, A^{-1} = H (A H)^{-1}).
 * GA = -GB X^T, n x n, ldga >= n; GB, X: n x nrhs (ldgb, ldx >= nrhs),
 * 1 <= nrhs <= 64.  All device pointers; GA may not alias GB or X.  Enqueued
 * on hip_stream, which is synchronised before returning. */
rmge_status rmge_grad_A(const double *GB, int64_t ldgb, const double *X, int64_t ldx, int64_t n,
                        int64_t nrhs, double *GA, int64_t ldga, void *hip_stream);

/* Factor statistics.  min_abs_pivot and growth are computed on the device at
 * the first call (one pass over M's diagonal and U) and cached. */
rmge_status rmge_factor_stats_get(const rmge_factors *f, rmge_factor_stats *s);

/* The phase times of the last factorization (the ms_* fields of
 * rmge_factor_stats, recorded by HIP events on the handle's stream), without
 * the device pass rmge_factor_stats_get makes for the growth: ms3[0] drawing H
 * (and rounding A), ms3[1] the product M = A H, ms3[2] the elimination.  Host
 * only; ms3 is a host array of 3 doubles.  EINVAL on a null argument. */
rmge_status rmge_factor_times(const rmge_factors *f, double *ms3);

/* Copy the packed factors (unit L strictly below the diagonal, U on and above)
 * into LU (device, n x n, ld >= n), converted to FP64.  Pivoted handles:
 * L U = P M, rows in the order of rmge_factors_perm. */
rmge_status rmge_factors_lu(const rmge_factors *f, double *LU, int64_t ld);

/* The row order of the factors: perm[t] = the row of M = A H stored at row t
 * (the identity without pivoting).  perm: device, n int32 values. */
rmge_status rmge_factors_perm(const rmge_factors *f, int32_t *perm);

/* The multiplier's random parameters as drawn by the library: kind GAUSSIAN
 * gives n*n values (G row-major), CIRCULANT n (c), TOEPLITZ 2n-1 (tau, with
 * tau[0..n-1] = t_0..t_{n-1} and tau[n-1+d] = t_{-d}).  out: device, FP64. */
rmge_status rmge_multiplier_params(int32_t kind, int64_t n, uint64_t seed, double *out,
                                   void *hip_stream);

/* Number of parameters rmge_multiplier_params writes (0 for NONE or bad kind). */
int64_t rmge_param_count(int32_t kind, int64_t n);

/* M = A H in FP64 (the preprocessing product alone): dense MFMA product for
 * GAUSSIAN, FFT correlation for CIRCULANT and TOEPLITZ, copy for NONE.
 * A, M: device n x n, lda, ldm >= n; M may not alias A. */
rmge_status rmge_precondition(const double *A, int64_t n, int64_t lda, int32_t kind,
                              uint64_t seed, double *M, int64_t ldm, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): M = A H
 * exactly as rmge_precondition computes it (the same kernels, so the same
 * values), with the multiplier's workspace in a fixed library-owned device
 * array of 8 MiB per GPU instead of an allocation.  It calls no hipMalloc,
 * hipFree or allocating library routine.  Sizes: NONE, CIRCULANT and
 * TOEPLITZ for every n rmge_precondition accepts (at most 0.7 MiB of
 * workspace); GAUSSIAN only while n * n doubles fit (n <= 1024); larger
 * sizes return RMGE_EINVAL.  The work is only enqueued on hip_stream (no
 * synchronisation; launch errors are returned).  Every call on one GPU uses
 * that GPU's one array, so calls whose work overlaps on one GPU (other
 * streams or threads, before the previous call's work has finished) race and
 * give undefined M; calls on one stream are ordered.  The array keeps the
 * last call's contents; every value a call reads is first written by it. */
rmge_status rmge_precondition_noalloc(const double *A, int64_t n, int64_t lda, int32_t kind,
                                      uint64_t seed, double *M, int64_t ldm, void *hip_stream);

void rmge_destroy(rmge_factors *f);

const char *rmge_status_string(int32_t s);

/* Library version as major*10000 + minor*100 + patch. */
int32_t rmge_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RMGE_H */
