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
