/*
 * rmge_oracle.c -- plain, slow, FP64 CPU oracle for random-multiplier GENP.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference that the GPU library
 * is checked against.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant with the GPU library; the two implement the same written
 * random-number specification independently.
 *
 * What it computes (Pan, Qian, Yan, "Random multipliers numerically stabilize
 * Gaussian and block Gaussian elimination", arXiv:1406.5802):
 *   1. a random multiplier H: Gaussian (Definition defrndm), circulant with a
 *      Gaussian first column (Section 6, definition of C and the "Gaussian
 *      circulant" remark after Theorem thcpw), Toeplitz (a leading block of a
 *      larger random circulant, Section 1.1 and Remark remsrtft) or a random
 *      unitary circulant (Section 6, Example exunc; real orthogonal here);
 *   2. the preprocessed matrix M = A H (Fact faprepr, post-multiplication);
 *   3. Gaussian elimination with no pivoting on M (Section 3: the complete
 *      recursive factorization with k = 1, eq. eqgenp), stopping at the first
 *      vanishing pivot (Corollary corec); or block Gaussian elimination whose
 *      recursion stops at small diagonal blocks that are handed to a black-box
 *      method (Section 3, after eq. eqgenpin), here Gaussian elimination with
 *      partial pivoting confined to each such block;
 *   4. y = U^{-1} L^{-1} b and x = H y (Fact faprepr);
 *   5. iterative refinement steps r = b - A x, x += H U^{-1} L^{-1} r
 *      (Section 8.1 protocol: one refinement step);
 *   6. the adjoint solve A^{-T} w = L^{-T} U^{-T} H^T w (Fact faprepr,
 *      transposed).
 *
 * Everything is plain loops in IEEE double, in the order the definitions
 * state.  No blocking, no FFT, no reordering of any single element's sum.
 * OpenMP only distributes independent rows over threads; it never changes the
 * arithmetic performed for an element.
 *
 * Matrices are row-major, n x n, leading dimension n, unless stated.
 * Right-hand sides B and solutions X are n x nrhs row-major.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel      */
/* random numbers: as easy as 1, 2, 3", SC'11), uniform doubles, Box-Muller. */
/* ------------------------------------------------------------------------ */

/* Round multipliers and Weyl key increments of Philox4x64 as published. */
static const uint64_t PHX_MUL0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PHX_MUL1 = 0xCA5A826395121157ULL;
static const uint64_t PHX_WEYL0 = 0x9E3779B97F4A7C15ULL; /* golden ratio */
static const uint64_t PHX_WEYL1 = 0xBB67AE8584CAA73BULL; /* sqrt(3) - 1 */

static void mul128(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

/* One Philox4x64 block with 10 rounds: out = philox(ctr, key). */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t hi0, lo0, hi1, lo1;
        mul128(PHX_MUL0, x0, &hi0, &lo0);
        mul128(PHX_MUL1, x2, &hi1, &lo1);
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += PHX_WEYL0;
        k1 += PHX_WEYL1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Random-number specification shared (as text, not code) with the GPU side:
 *   key     = (seed, 0)
 *   counter = (m, stream, 0, 0) for block m = 0, 1, 2, ...
 *   uniform u_j = ((w_j >> 12) + 0.5) * 2^-52, j = 0..3: exact in binary64 and
 *   strictly inside (0, 1)
 *   normals from Box-Muller on the pairs (u0, u1) and (u2, u3):
 *       z0 = sqrt(-2 ln u0) cos(2 pi u1),  z1 = sqrt(-2 ln u0) sin(2 pi u1)
 *       z2 = sqrt(-2 ln u2) cos(2 pi u3),  z3 = sqrt(-2 ln u2) sin(2 pi u3)
 *   element e of a stream is output (e mod 4) of block e / 4.
 * Streams: 1 = Gaussian multiplier G (element i*n + j is G[i][j]),
 *          2 = circulant first column c, 3 = Toeplitz parameters tau,
 *          4 = phases of the unitary circulant (uniforms, element j is phi_j). */
static void orc_block(uint64_t seed, uint64_t stream, uint64_t m, uint64_t w[4]) {
    uint64_t ctr[4] = {m, stream, 0, 0};
    uint64_t key[2] = {seed, 0};
    orc_philox4x64_10(ctr, key, w);
}

static double orc_word_to_uniform(uint64_t w) {
    return ((double)(w >> 12) + 0.5) * 0x1.0p-52;
}

void orc_uniforms(uint64_t seed, uint64_t stream, int64_t count, double *out) {
    for (int64_t e = 0; e < count; ++e) {
        uint64_t w[4];
        orc_block(seed, stream, (uint64_t)(e / 4), w);
        out[e] = orc_word_to_uniform(w[e % 4]);
    }
}

void orc_words(uint64_t seed, uint64_t stream, int64_t nblocks, uint64_t *out) {
    for (int64_t m = 0; m < nblocks; ++m) orc_block(seed, stream, (uint64_t)m, out + 4 * m);
}

/* Standard Gaussian variables (Definition defrndm: mean 0, variance 1). */
void orc_normals(uint64_t seed, uint64_t stream, int64_t count, double *out) {
    const double two_pi = 6.283185307179586476925286766559;
    int64_t nblocks = (count + 3) / 4;
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < nblocks; ++m) {
        uint64_t w[4];
        orc_block(seed, stream, (uint64_t)m, w);
        double u0 = orc_word_to_uniform(w[0]), u1 = orc_word_to_uniform(w[1]);
        double u2 = orc_word_to_uniform(w[2]), u3 = orc_word_to_uniform(w[3]);
        double r01 = sqrt(-2.0 * log(u0));
        double r23 = sqrt(-2.0 * log(u2));
        double z[4];
        z[0] = r01 * cos(two_pi * u1);
        z[1] = r01 * sin(two_pi * u1);
        z[2] = r23 * cos(two_pi * u3);
        z[3] = r23 * sin(two_pi * u3);
        for (int j = 0; j < 4; ++j) {
            int64_t e = 4 * m + j;
            if (e < count) out[e] = z[j];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Multipliers, written out as dense n x n matrices.                        */
/* ------------------------------------------------------------------------ */

enum { ORC_NONE = 0, ORC_GAUSSIAN = 1, ORC_CIRCULANT = 2, ORC_TOEPLITZ = 3,
       ORC_UNITARY_CIRCULANT = 4 };

/* Number of parameters that define each multiplier kind (for the unitary
 * circulant: its first column, computed from n random phases). */
int64_t orc_param_count(int kind, int64_t n) {
    switch (kind) {
    case ORC_GAUSSIAN: return n * n;
    case ORC_CIRCULANT: return n;
    case ORC_TOEPLITZ: return 2 * n - 1;
    case ORC_UNITARY_CIRCULANT: return n;
    default: return 0;
    }
}

/* The spectrum u of the random unitary circulant (Example exunc, step (i)),
 * made conjugate-symmetric so that the circulant is real: from n uniforms
 * phi_0..phi_{n-1} of stream 4,
 *   u_j = exp(2 pi i phi_j) and u_{n-j} = conj(u_j) for 0 < j < n/2,
 *   u_0 = +1 if phi_0 < 1/2 else -1, and for even n u_{n/2} = +1 if
 *   phi_{n/2} < 1/2 else -1 (the two entries that must be real);
 * phi_j for j > n/2 are drawn and not used.  Every |u_j| = 1. */
void orc_unitary_spectrum(int64_t n, uint64_t seed, double *ure, double *uim) {
    const double two_pi = 6.283185307179586476925286766559;
    double *phi = (double *)malloc(sizeof(double) * (size_t)n);
    orc_uniforms(seed, (uint64_t)ORC_UNITARY_CIRCULANT, n, phi);
    for (int64_t j = 0; j < n; ++j) { ure[j] = 0.0; uim[j] = 0.0; }
    ure[0] = phi[0] < 0.5 ? 1.0 : -1.0;
    for (int64_t j = 1; 2 * j < n; ++j) {
        ure[j] = cos(two_pi * phi[j]);
        uim[j] = sin(two_pi * phi[j]);
        ure[n - j] = ure[j];
        uim[n - j] = -uim[j];
    }
    if (n % 2 == 0 && n >= 2) ure[n / 2] = phi[n / 2] < 0.5 ? 1.0 : -1.0;
    free(phi);
}

/* First column c = Omega^{-1} u of the unitary circulant (Example exunc,
 * step (ii)), with Omega = (w^{jk}), w = exp(2 pi i / n) and
 * Omega^{-1} = Omega^H / n (Section 6): c_k = (1/n) sum_j u_j w^{-jk}, by
 * the plain O(n^2) sum.  w^{-jk} is taken as w^{-(jk mod n)} (w^n = 1), which
 * keeps the cosine's argument below 2 pi.  The imaginary parts cancel for a
 * conjugate-symmetric u; their largest magnitude is returned in *imag_max. */
void orc_unitary_column(int64_t n, const double *ure, const double *uim, double *c,
                        double *imag_max) {
    const double two_pi = 6.283185307179586476925286766559;
    double worst = 0.0;
#pragma omp parallel for schedule(static) reduction(max : worst)
    for (int64_t k = 0; k < n; ++k) {
        double sre = 0.0, sim = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const int64_t t = (j * k) % n;
            const double ang = -two_pi * (double)t / (double)n;
            const double wr = cos(ang), wi = sin(ang);
            sre += ure[j] * wr - uim[j] * wi;
            sim += ure[j] * wi + uim[j] * wr;
        }
        c[k] = sre / (double)n;
        if (fabs(sim / (double)n) > worst) worst = fabs(sim / (double)n);
    }
    if (imag_max) *imag_max = worst;
}

/* The parameters of the multiplier: G row-major, c, tau, or the unitary
 * circulant's first column. */
int orc_multiplier_params(int kind, int64_t n, uint64_t seed, double *p) {
    if (kind < ORC_GAUSSIAN || kind > ORC_UNITARY_CIRCULANT) return 1;
    if (kind == ORC_UNITARY_CIRCULANT) {
        double *ure = (double *)malloc(sizeof(double) * (size_t)n);
        double *uim = (double *)malloc(sizeof(double) * (size_t)n);
        orc_unitary_spectrum(n, seed, ure, uim);
        orc_unitary_column(n, ure, uim, p, NULL);
        free(ure);
        free(uim);
        return 0;
    }
    orc_normals(seed, (uint64_t)kind, orc_param_count(kind, n), p);
    return 0;
}

/* Dense H from its parameters.
 *   GAUSSIAN : H = G.
 *   CIRCULANT, UNITARY_CIRCULANT: H[i][j] = c[(i - j) mod n]  (Section 6,
 *              definition of C).
 *   TOEPLITZ : H[i][j] = t_{i-j}, with tau[0..n-1] = t_0..t_{n-1} (first column)
 *              and tau[n-1+d] = t_{-d} for d = 1..n-1 (first row).  This is the
 *              leading n x n block of a circulant of size 2n-1 whose first column
 *              is (t_0..t_{n-1}, t_{-(n-1)}..t_{-1}).
 *   NONE     : H = I (plain GENP, used to show breakdown). */
int orc_multiplier_dense(int kind, int64_t n, const double *p, double *H) {
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            double v;
            if (kind == ORC_NONE) {
                v = (i == j) ? 1.0 : 0.0;
            } else if (kind == ORC_GAUSSIAN) {
                v = p[i * n + j];
            } else if (kind == ORC_CIRCULANT || kind == ORC_UNITARY_CIRCULANT) {
                int64_t d = ((i - j) % n + n) % n;
                v = p[d];
            } else if (kind == ORC_TOEPLITZ) {
                int64_t d = i - j;
                v = (d >= 0) ? p[d] : p[n - 1 + (-d)];
            } else {
                return 1;
            }
            H[i * n + j] = v;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Dense products, plain i-k-j loops.                                       */
/* ------------------------------------------------------------------------ */

/* C (m x p) = A (m x q) * B (q x p), all row-major, contiguous. */
void orc_matmul(int64_t m, int64_t q, int64_t p, const double *A, const double *B, double *C) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        double *ci = C + i * p;
        for (int64_t j = 0; j < p; ++j) ci[j] = 0.0;
        for (int64_t k = 0; k < q; ++k) {
            double a = A[i * q + k];
            const double *bk = B + k * p;
            for (int64_t j = 0; j < p; ++j) ci[j] += a * bk[j];
        }
    }
}

/* y (n x nrhs) = H (n x n) * x (n x nrhs). */
static void orc_apply(int64_t n, int64_t nrhs, const double *H, const double *x, double *y) {
    orc_matmul(n, n, nrhs, H, x, y);
}

/* y (n x nrhs) = H^T (n x n) * x (n x nrhs). */
static void orc_apply_t(int64_t n, int64_t nrhs, const double *H, const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t r = 0; r < nrhs; ++r) {
            double s = 0.0;
            for (int64_t i = 0; i < n; ++i) s += H[i * n + j] * x[i * nrhs + r];
            y[j * nrhs + r] = s;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* GENP: Gaussian elimination with no pivoting, in place.                   */
/* ------------------------------------------------------------------------ */

/* Status codes (oracle-private; the GPU library has its own). */
enum { ORC_OK = 0, ORC_ZERO_PIVOT = 4, ORC_NONFINITE = 5 };

/* Right-looking elimination of one column at a time: the complete recursive
 * factorization of eq. eqgenp with pivot blocks of size 1 (Section 3).  After
 * the call, the strictly lower part of M holds the unit lower factor L (the
 * multipliers D B^{-1} of each step) and the upper part holds U.
 * *info is the 0-based index of the first pivot that is exactly zero or not
 * finite, or -1.  By Corollary corec a zero pivot occurs iff M is not strongly
 * nonsingular; elimination stops there. */
int orc_genp(int64_t n, double *M, int64_t *info) {
    *info = -1;
    for (int64_t k = 0; k < n; ++k) {
        double p = M[k * n + k];
        if (p == 0.0) { *info = k; return ORC_ZERO_PIVOT; }
        if (!isfinite(p)) { *info = k; return ORC_NONFINITE; }
#pragma omp parallel for schedule(static)
        for (int64_t i = k + 1; i < n; ++i) {
            double l = M[i * n + k] / p;
            M[i * n + k] = l;
            for (int64_t j = k + 1; j < n; ++j) M[i * n + j] -= l * M[k * n + j];
        }
    }
    return ORC_OK;
}

/* Block Gaussian elimination in which the recursion of eq. eqgenp stops at
 * the diagonal blocks [ends[q-1], ends[q]) (ends[-1] = 0, ends strictly
 * increasing, ends[nblk-1] = n), each handed to a black-box method (Section 3,
 * after eq. eqgenpin): here Gaussian elimination with partial pivoting confined
 * to that block.  For column k in block [s, e) the pivot is the entry of
 * largest magnitude among rows k .. e-1 of the current matrix (ties: the
 * smallest original row index), whole rows are exchanged, and every row below
 * k is eliminated.  Rows never move between blocks, so the leading block of
 * each block boundary is the same as without pivoting and the Schur
 * complements at the boundaries are those of eq. eqgenp.  The partition is the
 * caller's: any partition gives the same Schur complements at its boundaries.
 * Result: P M = L U with perm[t] = the original index of the row stored at t.
 * *info: first column whose candidates are all exactly zero (the leading block
 * at that boundary is singular), or a non-finite pivot; -1 otherwise.
 * Returns 1 (and leaves M untouched) if `ends` is not a valid partition. */
int orc_genp_local(int64_t n, int64_t nblk, const int64_t *ends, double *M, int64_t *perm,
                   int64_t *info) {
    *info = -1;
    if (nblk < 1 || ends[nblk - 1] != n) return 1;
    for (int64_t q = 0; q < nblk; ++q)
        if (ends[q] <= (q ? ends[q - 1] : 0)) return 1;
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int64_t q = 0;
    for (int64_t k = 0; k < n; ++k) {
        while (ends[q] <= k) ++q;
        int64_t we = ends[q], r = k;
        for (int64_t i = k + 1; i < we; ++i) {
            double a = fabs(M[i * n + k]), best = fabs(M[r * n + k]);
            if (a > best || (a == best && perm[i] < perm[r])) r = i;
        }
        if (r != k) {
            memcpy(tmp, M + r * n, sizeof(double) * (size_t)n);
            memcpy(M + r * n, M + k * n, sizeof(double) * (size_t)n);
            memcpy(M + k * n, tmp, sizeof(double) * (size_t)n);
            int64_t t = perm[r]; perm[r] = perm[k]; perm[k] = t;
        }
        double p = M[k * n + k];
        if (p == 0.0) { *info = k; free(tmp); return ORC_ZERO_PIVOT; }
        if (!isfinite(p)) { *info = k; free(tmp); return ORC_NONFINITE; }
#pragma omp parallel for schedule(static)
        for (int64_t i = k + 1; i < n; ++i) {
            double l = M[i * n + k] / p;
            M[i * n + k] = l;
            for (int64_t j = k + 1; j < n; ++j) M[i * n + j] -= l * M[k * n + j];
        }
    }
    free(tmp);
    return ORC_OK;
}

/* Solve L z = b in place (L unit lower, stored strictly below the diagonal). */
static void orc_lower_unit_solve(int64_t n, int64_t nrhs, const double *LU, double *z) {
    for (int64_t i = 0; i < n; ++i)
        for (int64_t r = 0; r < nrhs; ++r) {
            double s = z[i * nrhs + r];
            for (int64_t j = 0; j < i; ++j) s -= LU[i * n + j] * z[j * nrhs + r];
            z[i * nrhs + r] = s;
        }
}

/* Solve U z = b in place (U upper, diagonal included). */
static void orc_upper_solve(int64_t n, int64_t nrhs, const double *LU, double *z) {
    for (int64_t i = n - 1; i >= 0; --i)
        for (int64_t r = 0; r < nrhs; ++r) {
            double s = z[i * nrhs + r];
            for (int64_t j = i + 1; j < n; ++j) s -= LU[i * n + j] * z[j * nrhs + r];
            z[i * nrhs + r] = s / LU[i * n + i];
        }
}

/* Solve U^T z = b in place (U^T lower, non-unit). */
static void orc_upper_t_solve(int64_t n, int64_t nrhs, const double *LU, double *z) {
    for (int64_t i = 0; i < n; ++i)
        for (int64_t r = 0; r < nrhs; ++r) {
            double s = z[i * nrhs + r];
            for (int64_t j = 0; j < i; ++j) s -= LU[j * n + i] * z[j * nrhs + r];
            z[i * nrhs + r] = s / LU[i * n + i];
        }
}

/* Solve L^T z = b in place (L^T upper, unit diagonal). */
static void orc_lower_unit_t_solve(int64_t n, int64_t nrhs, const double *LU, double *z) {
    for (int64_t i = n - 1; i >= 0; --i)
        for (int64_t r = 0; r < nrhs; ++r) {
            double s = z[i * nrhs + r];
            for (int64_t j = i + 1; j < n; ++j) s -= LU[j * n + i] * z[j * nrhs + r];
            z[i * nrhs + r] = s;
        }
}

/* ------------------------------------------------------------------------ */
/* Error measures.                                                          */
/* ------------------------------------------------------------------------ */

/* Normwise backward error on the ORIGINAL A, max over right-hand sides:
 *   eta = ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf)
 * and the paper's relative residual ||A x - b|| / ||b|| in the 2-norm of each
 * vector (Section 8.1), max over right-hand sides. */
void orc_errors(int64_t n, int64_t nrhs, const double *A, const double *B, const double *X,
                double *eta, double *relres) {
    double anorm = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) s += fabs(A[i * n + j]);
        if (s > anorm) anorm = s;
    }
    double eta_max = 0.0, rel_max = 0.0;
    for (int64_t r = 0; r < nrhs; ++r) {
        double rinf = 0.0, xinf = 0.0, binf = 0.0, r2 = 0.0, b2 = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double s = B[i * nrhs + r];
            for (int64_t j = 0; j < n; ++j) s -= A[i * n + j] * X[j * nrhs + r];
            rinf = fmax(rinf, fabs(s));
            r2 += s * s;
            xinf = fmax(xinf, fabs(X[i * nrhs + r]));
            binf = fmax(binf, fabs(B[i * nrhs + r]));
            b2 += B[i * nrhs + r] * B[i * nrhs + r];
        }
        double e = rinf / (anorm * xinf + binf);
        double q = sqrt(r2) / sqrt(b2);
        if (e > eta_max || isnan(e)) eta_max = e;
        if (q > rel_max || isnan(q)) rel_max = q;
    }
    *eta = eta_max;
    *relres = rel_max;
}

/* ------------------------------------------------------------------------ */
/* The whole method.                                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t info;         /* first zero / non-finite pivot, or -1 */
    int32_t status;       /* ORC_OK, ORC_ZERO_PIVOT or ORC_NONFINITE */
    int32_t steps;        /* refinement steps performed */
    double eta[17];       /* eta after 0, 1, ... refinement steps */
    double relres[17];    /* the paper's relative residual, same indexing */
    double min_abs_pivot; /* min |u_kk| */
    double growth;        /* max |U| / max |M| */
} orc_stats;

/* Factor: M = A H, then GENP on M (nblk == 0), or the locally pivoted block
 * elimination of orc_genp_local with the diagonal blocks ending at ends[0 ..
 * nblk) (perm receives the row order).  H (n x n), LU (n x n) are outputs;
 * perm (n) and ends may be NULL when nblk == 0. */
int orc_factor_ex(int64_t n, const double *A, int kind, uint64_t seed, int64_t nblk,
                  const int64_t *ends, double *H, double *LU, int64_t *perm, orc_stats *st) {
    memset(st, 0, sizeof(*st));
    if (kind == ORC_NONE) {
        orc_multiplier_dense(kind, n, NULL, H);
    } else {
        double *p = (double *)malloc(sizeof(double) * (size_t)orc_param_count(kind, n));
        orc_multiplier_params(kind, n, seed, p);
        orc_multiplier_dense(kind, n, p, H);
        free(p);
    }
    orc_matmul(n, n, n, A, H, LU); /* M = A H  (Fact faprepr) */
    double mmax = 0.0;
    for (int64_t e = 0; e < n * n; ++e) mmax = fmax(mmax, fabs(LU[e]));
    int rc = nblk > 0 ? orc_genp_local(n, nblk, ends, LU, perm, &st->info)
                      : orc_genp(n, LU, &st->info);
    st->status = rc;
    if (rc == ORC_OK) {
        double umax = 0.0, pmin = INFINITY;
        for (int64_t i = 0; i < n; ++i) {
            pmin = fmin(pmin, fabs(LU[i * n + i]));
            for (int64_t j = i; j < n; ++j) umax = fmax(umax, fabs(LU[i * n + j]));
        }
        st->min_abs_pivot = pmin;
        st->growth = umax / mmax;
    }
    return rc;
}

int orc_factor(int64_t n, const double *A, int kind, uint64_t seed, double *H, double *LU,
               orc_stats *st) {
    return orc_factor_ex(n, A, kind, seed, 0, NULL, H, LU, NULL, st);
}

/* z = H U^{-1} L^{-1} P v : one application of the preprocessed inverse
 * ((P v)[t] = v[perm[t]]; perm NULL means P = I). */
static void orc_apply_inverse(int64_t n, int64_t nrhs, const double *H, const double *LU,
                              const int64_t *perm, const double *v, double *z, double *tmp) {
    if (perm) {
        for (int64_t t = 0; t < n; ++t)
            memcpy(tmp + t * nrhs, v + perm[t] * nrhs, sizeof(double) * (size_t)nrhs);
    } else {
        memcpy(tmp, v, sizeof(double) * (size_t)(n * nrhs));
    }
    orc_lower_unit_solve(n, nrhs, LU, tmp);
    orc_upper_solve(n, nrhs, LU, tmp);
    orc_apply(n, nrhs, H, tmp, z);
}

/* Solve A X = B through A H Y = B, X = H Y, then `refine` refinement steps.
 * Records eta and relres after each stage in st. */
int orc_solve(int64_t n, int64_t nrhs, const double *A, const double *H, const double *LU,
              const int64_t *perm, const double *B, double *X, int refine, orc_stats *st) {
    if (refine > 16) refine = 16;
    size_t sz = sizeof(double) * (size_t)(n * nrhs);
    double *tmp = (double *)malloc(sz), *r = (double *)malloc(sz), *d = (double *)malloc(sz);
    orc_apply_inverse(n, nrhs, H, LU, perm, B, X, tmp);
    orc_errors(n, nrhs, A, B, X, &st->eta[0], &st->relres[0]);
    for (int s = 1; s <= refine; ++s) {
        /* r = B - A X in FP64 */
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t c = 0; c < nrhs; ++c) {
                double acc = B[i * nrhs + c];
                for (int64_t j = 0; j < n; ++j) acc -= A[i * n + j] * X[j * nrhs + c];
                r[i * nrhs + c] = acc;
            }
        orc_apply_inverse(n, nrhs, H, LU, perm, r, d, tmp);
        for (int64_t e = 0; e < n * nrhs; ++e) X[e] += d[e];
        orc_errors(n, nrhs, A, B, X, &st->eta[s], &st->relres[s]);
    }
    st->steps = refine;
    free(tmp); free(r); free(d);
    return 0;
}

/* Adjoint solve Y = A^{-T} W.  From A^{-1} = H (A H)^{-1} (Fact faprepr) and
 * P A H = L U: A^{-T} = P^T L^{-T} U^{-T} H^T (perm NULL means P = I). */
int orc_solve_adjoint(int64_t n, int64_t nrhs, const double *H, const double *LU,
                      const int64_t *perm, const double *W, double *Y) {
    size_t sz = sizeof(double) * (size_t)(n * nrhs);
    double *g = (double *)malloc(sz > 0 ? sz : 1);
    orc_apply_t(n, nrhs, H, W, g);
    orc_upper_t_solve(n, nrhs, LU, g);
    orc_lower_unit_t_solve(n, nrhs, LU, g);
    if (perm) {
        for (int64_t t = 0; t < n; ++t)
            memcpy(Y + perm[t] * nrhs, g + t * nrhs, sizeof(double) * (size_t)nrhs);
    } else {
        memcpy(Y, g, sz);
    }
    free(g);
    return 0;
}

/* Gradient of the loss sum(w .* x) with x = A^{-1} b:
 *   grad_b = A^{-T} w,  grad_A = -grad_b x^T  (n x n, summed over nrhs). */
void orc_grad_A(int64_t n, int64_t nrhs, const double *gb, const double *X, double *gA) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double s = 0.0;
            for (int64_t r = 0; r < nrhs; ++r) s += gb[i * nrhs + r] * X[j * nrhs + r];
            gA[i * n + j] = -s;
        }
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the rows the OpenMP loops distribute (the arithmetic of each
 * element does not depend on it). */
void orc_set_num_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}
