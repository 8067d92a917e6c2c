"""Pins for the oracle's GENP (Section 3, eq. eqgenp; Corollary corec; Theorem thnorms).

* On small integer matrices the FP64 LU equals the exact rational LU to within
  rounding, and the breakdown index is the exact one.
* Pivot identity: u_kk = det A^(k) / det A^(k-1) (from det A = det B det S,
  Corollary corec), with the leading minors computed by the Leibniz formula.
* Order independence (Section 3): block elimination with any pivot-block sizes
  that sum to k gives the same Schur complement, and it equals the trailing
  block of the oracle's partially eliminated matrix.
* Theorem thnorms bounds on |pivot| and 1/|pivot|.
"""
from fractions import Fraction

import numpy as np
import pytest

import workloads
from oracle import exact
from oracle import uniform_blocks
from partition import library_blocks, spans


def _strongly_nonsingular_int(n, seed):
    for s in range(seed, seed + 200):
        A = workloads.integer_matrix(n, s)
        minors = exact.leading_minors(exact.to_frac(A))
        if all(m != 0 for m in minors):
            return A
    raise RuntimeError("no strongly nonsingular draw")


@pytest.mark.parametrize("n,seed", [(2, 0), (3, 1), (5, 2), (6, 3), (7, 4)])
def test_lu_matches_exact_rationals(orc, n, seed):
    A = _strongly_nonsingular_int(n, seed)
    LU, rc, info = orc.genp(A)
    assert rc == orc.OK and info == -1
    ex, einfo = exact.genp(exact.to_frac(A))
    assert einfo == -1
    want = np.array([[float(v) for v in row] for row in ex])
    np.testing.assert_allclose(LU, want, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n,seed", [(4, 0), (6, 1), (7, 2)])
def test_pivots_are_minor_ratios(orc, n, seed):
    A = _strongly_nonsingular_int(n, seed)
    LU, rc, _ = orc.genp(A)
    minors = exact.leading_minors(exact.to_frac(A))
    prev = Fraction(1)
    for k in range(n):
        want = minors[k] / prev
        assert LU[k, k] == pytest.approx(float(want), rel=1e-12)
        prev = minors[k]


def test_breakdown_index_exact(orc):
    # leading 2x2 block singular, leading 1x1 and the whole matrix are not
    A = np.array([[1.0, 2.0, 0.0, 1.0],
                  [2.0, 4.0, 1.0, 0.0],
                  [0.0, 1.0, 3.0, 1.0],
                  [1.0, 0.0, 1.0, 2.0]])
    minors = exact.leading_minors(exact.to_frac(A))
    assert minors[0] != 0 and minors[1] == 0 and minors[3] != 0
    _, rc, info = orc.genp(A)
    assert rc == orc.ZERO_PIVOT and info == 1
    _, einfo = exact.genp(exact.to_frac(A))
    assert einfo == 1


def test_breakdown_case_zero_pivot_at_63(orc):
    A = workloads.breakdown_case(seed=0)
    f = orc.factor(A, orc.NONE, 0)
    assert f.status == orc.ZERO_PIVOT and f.info == 63
    assert f.LU[63, 63] == 0.0
    # not a zero pivot because A is singular: A itself is well conditioned
    assert np.linalg.cond(A) < 1e6


def test_nonfinite_pivot(orc):
    A = workloads.conditioned(8, 10.0, seed=1)
    A[3, 5] = np.nan
    _, rc, info = orc.genp(A)
    assert rc == orc.NONFINITE and info >= 3


@pytest.mark.parametrize("sizes", [[1, 1, 1, 1, 1], [2, 3], [3, 2], [5], [1, 4], [4, 1], [2, 2, 1]])
def test_block_order_independence_exact(sizes):
    A = exact.to_frac(_strongly_nonsingular_int(6, 7))
    ref = exact.block_schur_sequence(A, [1] * 6)  # GENP: Schur complements after 1, 2, ... steps
    got = exact.block_schur_sequence(A, sizes)
    k = 0
    for d, S in zip(sizes, got):
        k += d
        assert S == ref[k - 1]


def test_oracle_trailing_block_is_schur_complement(orc):
    A = _strongly_nonsingular_int(6, 9)
    Af = exact.to_frac(A)
    k = 3
    S = exact.block_schur_sequence(Af, [k, 6 - k])[0]
    # run the oracle's elimination on the leading k columns only: eliminate the
    # full matrix and rebuild the Schur complement from the factors.
    LU, rc, _ = orc.genp(A)
    L = np.tril(LU, -1) + np.eye(6)
    U = np.triu(LU)
    trailing = L[k:, k:] @ U[k:, k:]
    want = np.array([[float(v) for v in row] for row in S])
    np.testing.assert_allclose(trailing, want, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n,kind,seed", [(50, 1, 3), (97, 2, 4), (64, 3, 5), (128, 1, 6)])
def test_lu_reconstructs_AH(orc, n, kind, seed):
    A = workloads.conditioned(n, 1e3, seed)
    f = orc.factor(A, kind, seed)
    assert f.status == orc.OK
    L = np.tril(f.LU, -1) + np.eye(n)
    U = np.triu(f.LU)
    M = A @ f.H
    err = np.abs(L @ U - M).max()
    bound = 4 * n * np.finfo(float).eps * (np.abs(L) @ np.abs(U)).max()
    assert err <= bound


@pytest.mark.parametrize("seed", range(3))
def test_pivot_bounds_theorem_thnorms(orc, seed):
    n = 40
    M = workloads.conditioned(n, 50.0, seed) @ orc.multiplier(orc.GAUSSIAN, n, seed)
    LU, rc, _ = orc.genp(M)
    assert rc == orc.OK
    N = np.linalg.norm(M, 2)
    Nm = max(np.linalg.norm(np.linalg.inv(M[:j, :j]), 2) for j in range(1, n + 1))
    piv = np.abs(np.diag(LU))
    assert np.all(piv <= (N + Nm * N * N) * (1 + 1e-10))
    assert np.all(1.0 / piv <= Nm * (1 + 1e-8))


# ---------------------------------------------------------------------------
# Block elimination with partial pivoting confined to the small diagonal blocks
# (Section 3, after eq. eqgenpin: the recursion of eq. eqgenp may stop at small
# blocks that a black-box method handles).
# ---------------------------------------------------------------------------

def _windows(n, block):
    """Diagonal blocks [s, e) of width `block` (the last may be narrower)."""
    return spans(uniform_blocks(n, block))


def _lapack_perm(piv):
    perm = np.arange(len(piv))
    for i, p in enumerate(piv):
        perm[[i, p]] = perm[[p, i]]
    return perm


@pytest.mark.parametrize("n,seed", [(5, 0), (17, 1), (64, 2), (128, 3)])
def test_local_pivot_one_window_is_lapack_getrf(orc, n, seed):
    # one window covering the whole matrix: textbook partial pivoting (LAPACK getrf)
    import scipy.linalg as sl

    A = np.random.default_rng(seed).standard_normal((n, n))
    LU, perm, rc, info = orc.genp_local(A, [n])
    assert rc == orc.OK and info == -1
    lu, piv = sl.lu_factor(A)
    np.testing.assert_array_equal(perm, _lapack_perm(piv))
    np.testing.assert_allclose(LU, lu, rtol=0, atol=1e-12 * n)


@pytest.mark.parametrize("n,ends,seed", [(6, [2, 4, 6], 0), (7, [3, 6, 7], 1), (7, [7], 2),
                                         (6, [4, 6], 3), (7, [1, 4, 5, 7], 8)])
def test_local_pivot_products_of_pivots_are_leading_minors(orc, n, ends, seed):
    # Rows move only inside a window, so after each window [s, e) the product of
    # the pivots so far is +-det M^(e) (det A = det B det S, Corollary corec);
    # minors by the Leibniz formula.
    A = _strongly_nonsingular_int(n, seed)
    LU, perm, rc, info = orc.genp_local(A, ends)
    assert rc == orc.OK
    minors = exact.leading_minors(exact.to_frac(A))
    d = np.diag(LU)
    for s, e in spans(ends):
        assert abs(np.prod(d[:e])) == pytest.approx(abs(float(minors[e - 1])), rel=1e-11)
        # rows never leave their window
        assert sorted(perm[s:e]) == list(range(s, e))


@pytest.mark.parametrize("n,ends,seed", [(6, [2, 4, 6], 4), (7, [3, 6, 7], 5), (8, [4, 8], 6),
                                         (8, [1, 4, 6, 8], 7)])
def test_local_pivot_window_blocks_factor_exact_schur_complements(orc, n, ends, seed):
    # The diagonal block of window [s, e) factors the row-permuted leading block
    # of the exact Schur complement S(M^(s), M) (eq. eqgenp; exact rationals,
    # Gauss-Jordan inverses of the pivot blocks).
    A = _strongly_nonsingular_int(n, seed)
    LU, perm, rc, _ = orc.genp_local(A, ends)
    assert rc == orc.OK
    wins = spans(ends)
    schur = exact.block_schur_sequence(exact.to_frac(A), [e - s for s, e in wins])
    for idx, (s, e) in enumerate(wins):
        S = exact.to_frac(A) if idx == 0 else schur[idx - 1]
        w = e - s
        Bw = np.array([[float(v) for v in row[:w]] for row in S[:w]])
        Lw = np.tril(LU[s:e, s:e], -1) + np.eye(w)
        Uw = np.triu(LU[s:e, s:e])
        np.testing.assert_allclose(Lw @ Uw, Bw[perm[s:e] - s], rtol=1e-11, atol=1e-11)
        assert np.all(np.abs(np.tril(LU[s:e, s:e], -1)) <= 1.0 + 1e-15)


@pytest.mark.parametrize("n,block", [(64, 16), (100, 32), (300, 256), (257, 200)])
def test_local_pivot_reconstructs_PM(orc, n, block):
    # the library's partition (panels of `block`, wider than 128 cut once)
    A = np.random.default_rng(n).standard_normal((n, n))
    LU, perm, rc, _ = orc.genp_local(A, library_blocks(n, block))
    assert rc == orc.OK
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    np.testing.assert_allclose(L @ U, A[perm], rtol=0, atol=1e-11 * np.abs(A).max() * n)
    for s, e in spans(library_blocks(n, block)):
        assert sorted(perm[s:e]) == list(range(s, e))


def test_local_pivot_rejects_bad_partitions(orc):
    A = np.eye(4)
    for bad in ([], [2, 3], [3, 2, 4], [0, 4], [2, 2, 4]):
        with pytest.raises(ValueError):
            orc.genp_local(A, bad)


def test_local_pivot_block_one_is_genp(orc):
    A = _strongly_nonsingular_int(6, 7)
    LU1, perm, rc1, _ = orc.genp_local(A, uniform_blocks(6, 1))
    LU0, rc0, _ = orc.genp(A)
    assert rc1 == rc0 == orc.OK
    np.testing.assert_array_equal(perm, np.arange(6))
    np.testing.assert_array_equal(LU1, LU0)


def test_local_pivot_breakdown_and_rescue(orc):
    # leading 1x1 block zero: GENP breaks down at 0, a window of 2 pivots past it
    A = np.array([[0.0, 1.0, 2.0, 1.0],
                  [1.0, 0.0, 1.0, 3.0],
                  [2.0, 1.0, 0.0, 1.0],
                  [1.0, 2.0, 1.0, 1.0]])
    _, rc, info = orc.genp(A)
    assert rc == orc.ZERO_PIVOT and info == 0
    LU, perm, rc, info = orc.genp_local(A, [2, 4])
    assert rc == orc.OK and info == -1
    assert list(perm[:2]) == [1, 0]
    # leading 2x2 block singular: every window of 2 ends on an exactly zero pivot
    B = np.array([[1.0, 2.0, 0.0, 1.0],
                  [2.0, 4.0, 1.0, 0.0],
                  [0.0, 1.0, 3.0, 1.0],
                  [1.0, 0.0, 1.0, 2.0]])
    _, _, rc, info = orc.genp_local(B, [2, 4])
    assert rc == orc.ZERO_PIVOT and info == 1
    # ties: equal magnitudes choose the smaller original row index
    C = np.array([[1.0, 1.0], [-1.0, 2.0]])
    _, perm, rc, _ = orc.genp_local(C, [2])
    assert rc == orc.OK and list(perm) == [0, 1]
