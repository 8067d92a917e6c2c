"""Pins for the oracle's error measures and factor statistics.

* eta_inf = ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf) on the original A
  (the normwise backward error) and the paper's relative residual
  ||A x - b||_2 / ||b||_2 (Section 8.1), both maxed over right-hand sides:
  values worked out by hand on a 3 x 3 integer system whose residual is known,
  chosen so that ||A||_inf != ||A||_1, ||r||_2 != ||r||_inf and the largest
  value is not in the first or last column; and an independent numpy
  evaluation on a random case.
* growth = max |U| / max |M| and min |u_kk| (Theorem thnorms bounds the pivots):
  a hand-worked 3 x 3 elimination, exact rational elimination (including of
  the FP64 matrix M = A H itself, converted exactly to rationals), and pivots as
  ratios of Leibniz leading minors (Corollary corec: det A = det B det S).
* Each plausible slip in these formulas (1-norm for the inf-norm, inf-norm for
  the 2-norm, ||b||_2 in eta, growth over L as well as U or over A instead of
  M, signed pivots) is planted in a copy of the oracle's C source, built with
  gcc, and shown to break one of the pins above.
"""
import ctypes
import math
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import workloads
from oracle import exact

# ---- the hand-worked 3 x 3 system -------------------------------------------
# Row sums of |A|: 5, 6, 3 -> ||A||_inf = 6; column sums 5, 5, 4 -> ||A||_1 = 5.
A3 = np.array([[4.0, -1.0, 0.0],
               [1.0, 3.0, -2.0],
               [0.0, 1.0, 2.0]])
# column a: x = (1, -1, 2), A x = (5, -6, 3), b = (6, -6, 1): r = (1, 0, -2)
#   eta = 2 / (6*2 + 6) = 1/9;   relres = sqrt(5) / sqrt(73)
# column b: x = (0, 0, 10), A x = (0, -20, 20), b = (20, -20, 0): r = (20, 0, -20)
#   eta = 20 / (6*10 + 20) = 1/4;   relres = 20 sqrt(2) / (20 sqrt(2)) = 1
# column c: x = (0, 1, 0), A x = (-1, 3, 1), b = (-1, 4, 1): r = (0, 1, 0)
#   eta = 1 / (6*1 + 4) = 1/10;   relres = 1 / sqrt(18)
X3 = np.array([[1.0, 0.0, 0.0],
               [-1.0, 0.0, 1.0],
               [2.0, 10.0, 0.0]])
B3 = np.array([[6.0, 20.0, -1.0],
               [-6.0, -20.0, 4.0],
               [1.0, 0.0, 1.0]])
ETA3 = [1.0 / 9.0, 1.0 / 4.0, 1.0 / 10.0]
REL3 = [math.sqrt(5.0 / 73.0), 1.0, 1.0 / math.sqrt(18.0)]

# ---- the hand-worked elimination ----------------------------------------------
# M = [[2,1,1],[4,3,3],[8,7,9]]: l21 = 2, l31 = 4; rows become (0,1,1), (0,3,5);
# l32 = 3; last row (0,0,2).  U = [[2,1,1],[0,1,1],[0,0,2]]:
# max|U| = 2, max|M| = 9 -> growth 2/9; min |u_kk| = 1.  (max over L as well
# would be 4, over M would stay 9.)
M3 = np.array([[2.0, 1.0, 1.0], [4.0, 3.0, 3.0], [8.0, 7.0, 9.0]])
GROWTH3, MINPIV3 = 2.0 / 9.0, 1.0


def _strongly_nonsingular_int(n, seed):
    for s in range(seed, seed + 200):
        A = workloads.integer_matrix(n, s)
        if all(m != 0 for m in exact.leading_minors(exact.to_frac(A))):
            return A
    raise RuntimeError("no strongly nonsingular draw")


@pytest.mark.parametrize("col", [0, 1, 2])
def test_errors_single_rhs_hand_values(orc, col):
    eta, rel = orc.errors(A3, B3[:, col], X3[:, col])
    assert eta == pytest.approx(ETA3[col], rel=1e-15)
    assert rel == pytest.approx(REL3[col], rel=1e-15)


def test_errors_max_over_rhs_hand_values(orc):
    eta, rel = orc.errors(A3, B3, X3)
    assert eta == pytest.approx(max(ETA3), rel=1e-15)
    assert rel == pytest.approx(max(REL3), rel=1e-15)
    # the maximum sits in the middle column: neither the first nor the last decides
    assert np.argmax(ETA3) == 1 and np.argmax(REL3) == 1


def test_errors_match_numpy_definitions(orc):
    rng = np.random.default_rng(5)
    n, nrhs = 37, 4
    A = rng.standard_normal((n, n)) * rng.uniform(0.1, 10.0, size=(n, 1))
    X = rng.standard_normal((n, nrhs))
    B = A @ X + 1e-3 * rng.standard_normal((n, nrhs))
    eta, rel = orc.errors(A, B, X)
    R = B - A @ X
    anorm = np.linalg.norm(A, ord=np.inf)
    etas = [np.linalg.norm(R[:, r], np.inf)
            / (anorm * np.linalg.norm(X[:, r], np.inf) + np.linalg.norm(B[:, r], np.inf))
            for r in range(nrhs)]
    rels = [np.linalg.norm(R[:, r]) / np.linalg.norm(B[:, r]) for r in range(nrhs)]
    assert eta == pytest.approx(max(etas), rel=1e-10)
    assert rel == pytest.approx(max(rels), rel=1e-10)


def test_solve_reports_errors_on_the_original_A(orc):
    # the solve's recorded eta / relres are those of its returned X against the
    # ORIGINAL A (not M = A H)
    n = 40
    A = workloads.conditioned(n, 1e3, seed=3)
    B = workloads.rhs(n, 2, seed=4)
    f = orc.factor(A, orc.GAUSSIAN, 7)
    s = orc.solve(f, B, refine=1)
    e, r = orc.errors(A, B, s.X)
    assert s.eta[-1] == e and s.relres[-1] == r
    R = B - A @ s.X
    want = max(np.abs(R[:, c]).max() / (np.abs(A).sum(1).max() * np.abs(s.X[:, c]).max()
                                        + np.abs(B[:, c]).max()) for c in range(2))
    assert e == pytest.approx(want, rel=1e-6)


def test_growth_and_min_pivot_hand_values(orc):
    f = orc.factor(M3, orc.NONE, 0)
    assert f.status == orc.OK
    assert f.growth == pytest.approx(GROWTH3, rel=1e-15)
    assert f.min_abs_pivot == pytest.approx(MINPIV3, rel=1e-15)


@pytest.mark.parametrize("n,seed", [(4, 0), (5, 1), (6, 2), (7, 3)])
def test_growth_and_min_pivot_exact_rationals(orc, n, seed):
    A = _strongly_nonsingular_int(n, seed)
    f = orc.factor(A, orc.NONE, 0)
    assert f.status == orc.OK
    LU, info = exact.genp(exact.to_frac(A))
    assert info == -1
    umax = max(abs(LU[i][j]) for i in range(n) for j in range(i, n))
    assert f.growth == pytest.approx(float(umax / Fraction(int(np.abs(A).max()))), rel=1e-12)
    # pivots u_kk = det M^(k) / det M^(k-1), minors by the Leibniz formula
    minors = exact.leading_minors(exact.to_frac(A))
    piv = [minors[0]] + [minors[k] / minors[k - 1] for k in range(1, n)]
    assert f.min_abs_pivot == pytest.approx(float(min(abs(p) for p in piv)), rel=1e-12)


def test_growth_with_a_multiplier_is_relative_to_M(orc):
    # growth is max |U| over max |M| for M = A H: the FP64 matrix M converted
    # exactly to rationals and eliminated exactly
    n = 6
    A = _strongly_nonsingular_int(n, 11)
    f = orc.factor(A, orc.GAUSSIAN, 5)
    assert f.status == orc.OK
    M = orc.matmul(A, f.H)
    Mq = [[Fraction(float(v)) for v in row] for row in M]
    LU, info = exact.genp(Mq)
    assert info == -1
    umax = max(abs(LU[i][j]) for i in range(n) for j in range(i, n))
    mmax = max(abs(v) for row in Mq for v in row)
    assert f.growth == pytest.approx(float(umax / mmax), rel=1e-9)
    assert f.min_abs_pivot == pytest.approx(float(min(abs(LU[k][k]) for k in range(n))),
                                            rel=1e-9)


# ---- planted slips: each must break a pin above -------------------------------

_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                    "rmge_oracle.c")

MUTATIONS = {
    "anorm_one_norm": ("s += fabs(A[i * n + j]);", "s += fabs(A[j * n + i]);"),
    "relres_inf_norm": ("double q = sqrt(r2) / sqrt(b2);", "double q = rinf / binf;"),
    "eta_b_two_norm": ("double e = rinf / (anorm * xinf + binf);",
                       "double e = rinf / (anorm * xinf + sqrt(b2));"),
    "eta_x_two_norm": ("xinf = fmax(xinf, fabs(X[i * nrhs + r]));",
                       "xinf = sqrt(xinf * xinf + X[i * nrhs + r] * X[i * nrhs + r]);"),
    "growth_over_L_and_U": ("for (int64_t j = i; j < n; ++j) umax",
                            "for (int64_t j = 0; j < n; ++j) umax"),
    "growth_over_A": ("mmax = fmax(mmax, fabs(LU[e]));", "mmax = fmax(mmax, fabs(A[e]));"),
    "signed_pivots": ("pmin = fmin(pmin, fabs(LU[i * n + i]));",
                      "pmin = fmin(pmin, LU[i * n + i]);"),
}


class _Stats(ctypes.Structure):
    _fields_ = [("info", ctypes.c_int64), ("status", ctypes.c_int32),
                ("steps", ctypes.c_int32), ("eta", ctypes.c_double * 17),
                ("relres", ctypes.c_double * 17), ("min_abs_pivot", ctypes.c_double),
                ("growth", ctypes.c_double)]


def _build_mutant(tmp_path, name):
    old, new = MUTATIONS[name]
    src = open(_SRC).read()
    assert src.count(old) == 1, "mutation target not unique: %s" % name
    path = tmp_path / ("mut_%s.c" % name)
    path.write_text(src.replace(old, new))
    so = tmp_path / ("mut_%s.so" % name)
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off", str(path),
                    "-o", str(so), "-lm"], check=True)
    return ctypes.CDLL(str(so))


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _pins_hold(L):
    """Run the pins above against a (possibly mutated) oracle build; True if all hold."""
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    L.orc_errors.argtypes = [i64, i64, vp, vp, vp, vp, vp]
    L.orc_factor_ex.argtypes = [i64, vp, ctypes.c_int, ctypes.c_uint64, i64, vp, vp, vp, vp, vp]
    ok = True
    for col in range(3):
        A, B, X = (np.ascontiguousarray(m) for m in (A3, B3[:, col:col + 1], X3[:, col:col + 1]))
        e, r = ctypes.c_double(), ctypes.c_double()
        L.orc_errors(3, 1, _p(A), _p(B), _p(X), ctypes.byref(e), ctypes.byref(r))
        ok &= math.isclose(e.value, ETA3[col], rel_tol=1e-15)
        ok &= math.isclose(r.value, REL3[col], rel_tol=1e-15)
    cases = [(M3, 0, 0, GROWTH3, MINPIV3)]
    for n, seed in [(5, 1), (6, 2)]:
        A = _strongly_nonsingular_int(n, seed)
        LU, _ = exact.genp(exact.to_frac(A))
        g = max(abs(LU[i][j]) for i in range(n) for j in range(i, n)) / Fraction(
            int(np.abs(A).max()))
        cases.append((A, 0, 0, float(g), float(min(abs(LU[k][k]) for k in range(n)))))
    A6 = _strongly_nonsingular_int(6, 11)
    cases.append((A6, 1, 5, None, None))
    for A, kind, seed, g, p in cases:
        n = A.shape[0]
        A = np.ascontiguousarray(A, dtype=np.float64)
        H, LU, st = np.zeros((n, n)), np.zeros((n, n)), _Stats()
        L.orc_factor_ex(n, _p(A), kind, seed, 0, None, _p(H), _p(LU), None, ctypes.byref(st))
        if g is None:  # with a multiplier: exact elimination of M = A H
            Mq = [[Fraction(float(v)) for v in row] for row in A @ H]
            LUq, _ = exact.genp(Mq)
            g = float(max(abs(LUq[i][j]) for i in range(n) for j in range(i, n))
                      / max(abs(v) for row in Mq for v in row))
            p = float(min(abs(LUq[k][k]) for k in range(n)))
            ok &= math.isclose(st.growth, g, rel_tol=1e-9)
            ok &= math.isclose(st.min_abs_pivot, p, rel_tol=1e-9)
        else:
            ok &= math.isclose(st.growth, g, rel_tol=1e-12)
            ok &= math.isclose(st.min_abs_pivot, p, rel_tol=1e-12)
    return bool(ok)


def test_unmutated_oracle_passes_the_pin_harness(tmp_path):
    src = tmp_path / "orig.c"
    src.write_text(open(_SRC).read())
    so = tmp_path / "orig.so"
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off", str(src),
                    "-o", str(so), "-lm"], check=True)
    assert _pins_hold(ctypes.CDLL(str(so)))


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_slip_breaks_a_pin(tmp_path, name):
    assert not _pins_hold(_build_mutant(tmp_path, name)), name
