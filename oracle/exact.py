"""Exact-rational twin of the oracle -- TEST INFRASTRUCTURE ONLY.

Gaussian elimination with no pivoting (Section 3 of Pan, Qian, Yan,
arXiv:1406.5802: the complete recursive factorization of eq. eqgenp with unit
pivot blocks) and block elimination with arbitrary pivot-block sizes (the same
equation applied recursively with pivot blocks of several sizes), in
``fractions.Fraction`` for tiny integer inputs.  Used to pin the FP64 oracle:
on integer inputs small enough that no rounding can hide an error, the oracle's
L and U must equal the exact ones to within a few units of rounding, and the
breakdown index must be the same.
"""
from __future__ import annotations

from fractions import Fraction
from itertools import permutations


def to_frac(M):
    return [[Fraction(int(v)) if float(v).is_integer() else Fraction(v) for v in row] for row in M]


def matmul(A, B):
    n, q, p = len(A), len(B), len(B[0])
    return [[sum((A[i][k] * B[k][j] for k in range(q)), Fraction(0)) for j in range(p)]
            for i in range(n)]


def genp(M):
    """Unit pivot blocks.  Returns (LU packed, info) with info = first zero pivot or -1."""
    a = [row[:] for row in M]
    n = len(a)
    for k in range(n):
        p = a[k][k]
        if p == 0:
            return a, k
        for i in range(k + 1, n):
            a[i][k] = a[i][k] / p
            for j in range(k + 1, n):
                a[i][j] -= a[i][k] * a[k][j]
    return a, -1


def _inverse(B):
    """Gauss-Jordan inverse of a small nonsingular rational matrix (with row swaps:
    only used on a pivot block already known to be nonsingular)."""
    k = len(B)
    aug = [row[:] + [Fraction(int(i == j)) for j in range(k)] for i, row in enumerate(B)]
    for c in range(k):
        r = next(r for r in range(c, k) if aug[r][c] != 0)
        aug[c], aug[r] = aug[r], aug[c]
        piv = aug[c][c]
        aug[c] = [v / piv for v in aug[c]]
        for r in range(k):
            if r != c and aug[r][c] != 0:
                f = aug[r][c]
                aug[r] = [x - f * y for x, y in zip(aug[r], aug[c])]
    return [row[k:] for row in aug]


def _det(B):
    """Leibniz determinant: a sum over permutations, independent of elimination."""
    k = len(B)
    total = Fraction(0)
    for perm in permutations(range(k)):
        inv = sum(1 for i in range(k) for j in range(i + 1, k) if perm[i] > perm[j])
        term = Fraction(1)
        for i in range(k):
            term *= B[i][perm[i]]
        total += -term if inv % 2 else term
    return total


def leading_minors(M):
    """det of the leading k x k blocks, k = 1..n (brute force, Leibniz formula)."""
    return [_det([row[:k] for row in M[:k]]) for k in range(1, len(M) + 1)]


def block_schur_sequence(M, sizes):
    """Block elimination (eq. eqgenp) with pivot-block sizes ``sizes`` (summing to n).

    Returns the list of Schur complements S(A^(k), A) after each block step, or
    raises ZeroDivisionError if a pivot block is singular.  In exact arithmetic
    the Schur complement at position k does not depend on how the pivot sizes
    that sum to k are chosen (Section 3, discussion after eq. eqgenpin)."""
    a = [row[:] for row in M]
    out = []
    for d in sizes:
        if d == len(a):
            break
        B = [row[:d] for row in a[:d]]
        C = [row[d:] for row in a[:d]]
        D = [row[:d] for row in a[d:]]
        E = [row[d:] for row in a[d:]]
        if _det(B) == 0:
            raise ZeroDivisionError("singular pivot block")
        Binv = _inverse(B)
        DBC = matmul(matmul(D, Binv), C)
        a = [[E[i][j] - DBC[i][j] for j in range(len(E[0]))] for i in range(len(E))]
        out.append(a)
    return out
