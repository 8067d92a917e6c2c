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
    RMGE_MULT_TOEPLITZ = 3,  /* H[i][j] = t_{i-j}, 2n-1 i.i.d. N(0,1) parameters, FFT */
    /* Random unitary circulant (Section 6, Example exunc), real: H[i][j] =
     * c[(i-j) mod n] with c = Omega^{-1} u, Omega = (w^{jk}), w = e^{2 pi i/n},
     * and the spectrum u of unit modulus: u_j = e^{2 pi i phi_j} and
     * u_{n-j} = conj(u_j) for 0 < j < n/2, u_0 and (even n) u_{n/2} = +1 if
     * their phase is below 1/2, else -1; phi_j the uniforms of stream 4 of
     * the seed.  H is orthogonal (kappa(H) = 1, so kappa(A H) = kappa(A)).
     * Applied by FFT like RMGE_MULT_CIRCULANT. */
    RMGE_MULT_UNITARY_CIRCULANT = 4
} rmge_mult;

/* Precision of the factors L, U (and of the multiplier product M = A H).
 * Residuals and solution updates of refinement are always FP64. */
typedef enum {
    RMGE_F64 = 0,       /* FP64 MFMA */
    RMGE_F32 = 1,       /* FP32 MFMA with FP32 accumulation; refine in FP64 */
    RMGE_BF16 = 2,      /* BF16 factorization with FP32 accumulation: every bulk
                           Schur update (eq. eqgenp) of the trailing matrix runs on
                           the BF16 matrix cores with both operands rounded once
                           to BF16 (relative error up to 2^-9 each) and FP32
                           accumulation into the FP32 trailing matrix; the pivot
                           blocks, their solves and the updates of the next panel's
                           columns stay FP32 (as mixed-precision LU keeps its
                           panels in the higher precision).  Factors stored in
                           FP32; the product M = A H as for RMGE_F32_BF16X2.
                           Refine in FP64 (GMRES: the factors' error is of order
                           2^-9 times the growth). */
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
                           Other multiplier kinds: the FFT product in FP32 as for
                           RMGE_F32, and the same three-term BF16 Schur updates. */
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
 * column-by-column GENP).  On success *out receives a new handle.
 * Environment, read when a handle is created: RMGE_SIDE_CUS, the compute
 * units reserved for the look-ahead stream (default 32; 0: none, one shared
 * pool); RMGE_AUX_SCALE, the safety factor on their share of each wide Schur
 * update once the next pivot block is factored (default 1.0; 0: none). */
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
 * restart: 1..64.  tol > 0.  With one right-hand side st->iters counts its
 * inner iterations.  With 2..64 right-hand sides their Arnoldi processes
 * advance together (one preconditioner application, one product with op(A)
 * and one Gram-Schmidt pass a step for all of them; each column keeps its
 * own rotations and stops, keeping its iterate, once it meets the
 * estimate); st->iters then counts these joint steps and max_iters bounds
 * them.  More than 64 right-hand sides are refined one at a time.
 * st->eta_hist holds the worst eta at each outer check (first 17).  Returns
 * RMGE_NOT_CONVERGED if some right-hand side ends above tol.  Workspace,
 * kept by the handle: (2 restart + 2) n doubles for one right-hand side,
 * (2 restart + 2) n nrhs + 256 (restart + 1) nrhs doubles for several. */
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

/* The bulk Schur updates of the last factorization (eq. eqgenp: the trailing
 * block's update by the panel beyond the next pivot block, one launch per
 * step on the elimination's main stream): their summed device time in ms
 * (HIP events around each of those launches; 0 when the factorization had
 * more than 512 steps or broke down) and their algorithmic flops, sum of
 * 2 r w b over the steps (r trailing rows, w the columns the main stream's
 * launch updates: the r - b' beyond the next panel of width b', less the
 * last columns given to the reserved compute units; b this step's width).
 * Host only; no device work. */
rmge_status rmge_factor_update_time(const rmge_factors *f, double *ms, double *flops);

/* Copy the packed factors (unit L strictly below the diagonal, U on and above)
 * into LU (device, n x n, ld >= n), converted to FP64.  Pivoted handles:
 * L U = P M, rows in the order of rmge_factors_perm. */
rmge_status rmge_factors_lu(const rmge_factors *f, double *LU, int64_t ld);

/* The row order of the factors: perm[t] = the row of M = A H stored at row t
 * (the identity without pivoting).  perm: device, n int32 values. */
rmge_status rmge_factors_perm(const rmge_factors *f, int32_t *perm);

/* The multiplier's random parameters as drawn by the library: kind GAUSSIAN
 * gives n*n values (G row-major), CIRCULANT n (c), TOEPLITZ 2n-1 (tau, with
 * tau[0..n-1] = t_0..t_{n-1} and tau[n-1+d] = t_{-d}), UNITARY_CIRCULANT n
 * (its first column c, computed from the n phases).  out: device, FP64. */
rmge_status rmge_multiplier_params(int32_t kind, int64_t n, uint64_t seed, double *out,
                                   void *hip_stream);

/* Number of parameters rmge_multiplier_params writes (0 for NONE or bad kind). */
int64_t rmge_param_count(int32_t kind, int64_t n);

/* M = A H in FP64 (the preprocessing product alone): dense MFMA product for
 * GAUSSIAN, FFT correlation for CIRCULANT, TOEPLITZ and UNITARY_CIRCULANT,
 * copy for NONE.
 * A, M: device n x n, lda, ldm >= n; M may not alias A. */
rmge_status rmge_precondition(const double *A, int64_t n, int64_t lda, int32_t kind,
                              uint64_t seed, double *M, int64_t ldm, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): M = A H
 * exactly as rmge_precondition computes it (the same kernels, so the same
 * values), with the multiplier's workspace in a fixed library-owned device
 * array of 8 MiB per GPU instead of an allocation.  It calls no hipMalloc,
 * hipFree or allocating library routine.  Sizes: NONE and the FFT kinds
 * (CIRCULANT, TOEPLITZ, UNITARY_CIRCULANT) for every n rmge_precondition
 * accepts (at most 0.7 MiB of workspace); GAUSSIAN only while n * n doubles
 * fit (n <= 1024); larger sizes return RMGE_EINVAL.  The work is only enqueued on hip_stream (no
 * synchronisation; launch errors are returned).  Every call on one GPU uses
 * that GPU's one array, so calls whose work overlaps on one GPU (other
 * streams or threads, before the previous call's work has finished) race and
 * give undefined M; calls on one stream are ordered.  The array keeps the
 * last call's contents; every value a call reads is first written by it. */
rmge_status rmge_precondition_noalloc(const double *A, int64_t n, int64_t lda, int32_t kind,
                                      uint64_t seed, double *M, int64_t ldm, void *hip_stream);

/* One Schur-complement update of the elimination, C <- C - D E (eq. eqgenp:
 * the trailing block minus the product of the column below the pivot block
 * and the block row right of it, the pivot block's solves already applied),
 * in FP32, exactly as the factorization runs it for trailing blocks:
 * terms = 0: FP32 matrix cores; terms = 3: the three-term BF16 split of
 * RMGE_F32_BF16X2 (six BF16 products, FP32 accumulation); terms = 1: the BF16
 * update of RMGE_BF16 (operands rounded once to BF16).  D: M x K (ldd >= K),
 * E: K x N (lde >= N), C: M x N (ldc >= N), device FP32, row-major, C not
 * overlapping D or E; K <= 256.  Allocates its workspace, synchronises
 * hip_stream. */
rmge_status rmge_schur_update_f32(int64_t M, int64_t N, int64_t K, const float *D, int64_t ldd,
                                  const float *E, int64_t lde, float *C, int64_t ldc,
                                  int32_t terms, void *hip_stream);

/* ---------------------------------------------------------------------------
 * Batches: many independent systems A_s x_s = b_s of uneven order solved by
 * the method in one device-resident pass (Definition defrndm and Section 6 for
 * the multipliers, Fact faprepr, eq. eqgenp, Section 8.1 refinement).  Per
 * system: its multiplier H_s from its own seed (a dense Gaussian, or a
 * circulant with a Gaussian first column applied by FFT), M_s = A_s H_s in
 * FP32 (A rounded to FP32), block Gaussian elimination with no pivoting in
 * FP32 on the matrix cores with pivot blocks of nb columns (nb per size
 * bucket, see rmge_batch_tuning), then x_s = H_s U_s^{-1} L_s^{-1} b_s refined
 * in FP64 by restarted flexible GMRES preconditioned with the factors until
 * eta_s <= tol or max_iters inner iterations, eta the normwise backward error
 * ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf).  A system still above
 * tol then is solved again from FP64 factors of the same M_s = A_s H_s
 * (FP64 product, GENP with pivot blocks of 32, the same refinement), and its
 * result says so.  The systems are taken
 * largest first by persistent kernels; nothing is synchronised or allocated
 * while running, so a run can be captured into a HIP graph
 * (rmge_batch_graph_run does that itself).
 * ------------------------------------------------------------------------- */
typedef struct rmge_batch rmge_batch; /* opaque; owned by the library */

typedef struct {
    int32_t n;     /* order, 1 <= n <= 1024 */
    int32_t kind;  /* RMGE_MULT_GAUSSIAN or RMGE_MULT_CIRCULANT */
    uint64_t seed; /* the system's multiplier seed (the single-system generator) */
    int64_t a_off; /* element offset of A_s (n x n, row-major, ld = n) in the A buffer */
    int64_t v_off; /* element offset of b_s and x_s (n values each) in B and X */
} rmge_batch_system;

#define RMGE_BATCH_BUCKETS 5
/* Pivot-block width per size bucket (n <= 64, <= 128, <= 256, <= 512, <= 1024);
 * each 16, 32 or 64. */
typedef struct {
    int32_t nb[RMGE_BATCH_BUCKETS];
} rmge_batch_tuning;

/* Describe a batch.  systems: host array of count entries (copied).  tuning:
 * NULL for the defaults {32, 32, 32, 64, 64}.  restart: GMRES restart length,
 * 1..32.  max_iters: inner iterations per system.  Allocates the device
 * workspace (for every system: n^2 FP32 factors, n^2 doubles for FP64 factors
 * should it fall back, (2 restart + 1) n doubles; Gaussian: n^2 FP32 for G;
 * circulant: O(n)).  EINVAL on a bad entry. */
rmge_status rmge_batch_create(const rmge_batch_system *systems, int32_t count,
                              const rmge_batch_tuning *tuning, int32_t restart, int32_t max_iters,
                              rmge_batch **out);

/* Solve every system: A, B, X device FP64 buffers laid out as the systems'
 * offsets say (A never written; X may not overlap A or B).  Only enqueues work
 * on hip_stream: no synchronisation, no allocation.  tol > 0.  Systems whose
 * factorization meets a zero or non-finite pivot keep their X untouched. */
rmge_status rmge_batch_run(rmge_batch *b, const double *A, const double *B, double *X, double tol,
                           void *hip_stream);

/* As rmge_batch_run, with HIP events between the phases, synchronised:
 * ms4[0] drawing the multipliers and forming every M_s = A_s H_s, ms4[1] the
 * factorizations, ms4[2] the solves and refinement, ms4[3] the FP64 fallback
 * (host array of 4). */
rmge_status rmge_batch_run_timed(rmge_batch *b, const double *A, const double *B, double *X,
                                 double tol, void *hip_stream, double *ms4);

/* As rmge_batch_run, through a HIP graph: the first call (and any call with
 * other buffers or tol) captures the whole run into a graph on the library's
 * own stream; every call then launches that graph on hip_stream. */
rmge_status rmge_batch_graph_run(rmge_batch *b, const double *A, const double *B, double *X,
                                 double tol, void *hip_stream);

/* Per-system results of the last run, in the order of `systems` (host arrays
 * of count entries, each may be NULL): status (RMGE_OK, RMGE_ZERO_PIVOT,
 * RMGE_NONFINITE or RMGE_NOT_CONVERGED), final eta, eta of the unrefined
 * solution, inner iterations (both stages), the first zero / non-finite
 * pivot's index (-1 if none), and 1 where the system was solved again from
 * FP64 factors.  Synchronises hip_stream first. */
rmge_status rmge_batch_results(const rmge_batch *b, int32_t *status, double *eta, double *eta0,
                               int32_t *iters, int64_t *info, int32_t *fp64, void *hip_stream);

rmge_status rmge_batch_get_tuning(const rmge_batch *b, rmge_batch_tuning *t);
rmge_status rmge_batch_set_tuning(rmge_batch *b, const rmge_batch_tuning *t);

/* Autotuner: for each size bucket in turn, time the batch's factorization of
 * that bucket's systems (HIP events, after a warm-up run) with pivot blocks of
 * 16, 32 and 64 columns, the products redone before each timing, and keep the
 * fastest.  The chosen widths are applied to the batch and returned in *best;
 * ms_bucket (host, RMGE_BATCH_BUCKETS entries, may be NULL) receives the best
 * times (-1 for an empty bucket).  A: the systems' matrices. Synchronises. */
rmge_status rmge_batch_autotune(rmge_batch *b, const double *A, void *hip_stream,
                                rmge_batch_tuning *best, double *ms_bucket);

/* The packed FP32 factors of system `index` (in the order of `systems`) after
 * a run, converted to FP64 into LU (device, n x n, ld >= n): unit L strictly
 * below the diagonal, U on and above, L U = M_s = A_s H_s (A_s rounded to
 * FP32, H_s in FP32).  Synchronises hip_stream. */
rmge_status rmge_batch_factors_lu(const rmge_batch *b, int32_t index, double *LU, int64_t ld,
                                  void *hip_stream);

void rmge_batch_destroy(rmge_batch *b);

void rmge_destroy(rmge_factors *f);

const char *rmge_status_string(int32_t s);

/* Library version as major*10000 + minor*100 + patch. */
int32_t rmge_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RMGE_H */
