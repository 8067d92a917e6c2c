"""Pins for the oracle's solve, refinement and adjoint.

* Fact faprepr: A x = b is solved through A H y = b, x = H y; the solution is
  checked against LAPACK's pivoted solver (numpy) and, on tiny integer systems,
  against sympy's exact rational solve.
* Section 8.1: plain GENP fails on inputs with a singular leading block, and
  with a Gaussian multiplier plus one refinement step it is backward stable.
* The adjoint A^{-T} w = L^{-T} U^{-T} H^T w against numpy, and the gradient
  of sum(w * x) against central finite differences.
"""
import os

import numpy as np
import pytest
import sympy

import workloads
from partition import library_blocks

EPS = np.finfo(float).eps


@pytest.mark.parametrize("kind", [1, 2, 3])
@pytest.mark.parametrize("kappa", [1e2, 1e6])
def test_solution_matches_lapack(orc, kind, kappa):
    n = 96
    A = workloads.conditioned(n, kappa, seed=3)
    B = workloads.rhs(n, 3, seed=3)
    f = orc.factor(A, kind, seed=101)
    assert f.status == orc.OK
    s = orc.solve(f, B, refine=1)
    X = np.linalg.solve(A, B)
    rel = np.linalg.norm(s.X - X) / np.linalg.norm(X)
    assert rel <= max(1e-12, 8 * kappa * n * EPS)
    assert s.eta[-1] <= 1e-15


def test_exact_rational_solution(orc):
    n = 5
    A = workloads.integer_matrix(n, 3)
    b = workloads.integer_matrix(n, 4)[:, 0]
    x_exact = sympy.Matrix(A.astype(int).tolist()).LUsolve(sympy.Matrix(b.astype(int).tolist()))
    x_exact = np.array([float(v) for v in x_exact])
    for kind in (0, 1, 2, 3):
        f = orc.factor(A, kind, seed=7)
        if f.status != orc.OK:
            assert kind == 0  # only plain GENP may break down on a random integer matrix
            continue
        s = orc.solve(f, b, refine=2)
        np.testing.assert_allclose(s.X, x_exact, rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("seed", range(3))
def test_breakdown_case_preprocessed_is_stable(orc, seed):
    A = workloads.breakdown_case(seed)
    b = workloads.rhs(256, 1, seed)
    f0 = orc.factor(A, orc.NONE, 0)
    assert f0.status == orc.ZERO_PIVOT and f0.info == 63
    f = orc.factor(A, orc.GAUSSIAN, seed + 1000)
    assert f.status == orc.OK
    s = orc.solve(f, b, refine=1)
    assert min(s.eta) <= 1e-13
    assert s.eta[1] <= 1e-15


def _table(name, n, steps):
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.txt")
    for line in open(path):
        p = line.split()
        if p and p[0] == name and int(p[1]) == n and int(p[2]) == steps:
            return dict(mean=float(p[3]), max=float(p[4]), min=float(p[5]))
    raise KeyError((name, n, steps))


@pytest.mark.parametrize("n", [64, 128])
def test_paper_family_statistics(orc, n):
    """Section 8.1 family: distributional agreement with Table tab63 (orders of
    magnitude only -- per-instance values are not fixed by the paper)."""
    runs = 12
    rr0, rr1, plain = [], [], []
    for seed in range(runs):
        A = workloads.paper_e1(n, seed)
        b = workloads.rhs(n, 1, seed)
        f = orc.factor(A, orc.GAUSSIAN, seed)
        s = orc.solve(f, b, refine=1)
        rr0.append(s.relres[0])
        rr1.append(s.relres[1])
        g = orc.factor(A, orc.NONE, 0)
        if g.status == orc.OK:
            plain.append(orc.solve(g, b, refine=0).relres[0])
        else:
            plain.append(np.inf)
    t0, t1 = _table("tab63", n, 0), _table("tab63", n, 1)
    assert max(rr0) <= 100 * t0["max"]
    assert np.median(rr1) <= 100 * t1["mean"]
    assert max(rr1) <= 100 * t1["max"]
    # plain GENP: the paper saw relative residuals 1e-3 .. 1e2 (or outright failure)
    assert min(plain) >= 1e-6


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
def test_adjoint_matches_lapack(orc, kind):
    n = 70
    A = workloads.conditioned(n, 1e3, seed=5)
    W = workloads.rhs(n, 4, seed=6)
    f = orc.factor(A, kind, seed=8)
    Y = orc.solve_adjoint(f, W)
    want = np.linalg.solve(A.T, W)
    np.testing.assert_allclose(Y, want, rtol=0, atol=1e-9 * np.abs(want).max())


def test_gradient_central_differences(orc):
    n, nrhs = 24, 3
    A = workloads.conditioned(n, 30.0, seed=1)
    B = workloads.rhs(n, nrhs, seed=2)
    Wt = workloads.rhs(n, nrhs, seed=3)

    def loss(Am):
        f = orc.factor(Am, orc.TOEPLITZ, 5)
        return float(np.sum(Wt * orc.solve(f, B, refine=2).X))

    f = orc.factor(A, orc.TOEPLITZ, 5)
    X = orc.solve(f, B, refine=2).X
    gb = orc.solve_adjoint(f, Wt)
    gA = orc.grad_A(gb, X)
    rng = np.random.default_rng(0)
    h = 1e-6
    for _ in range(12):
        i, j = rng.integers(0, n, 2)
        Ap, Am = A.copy(), A.copy()
        Ap[i, j] += h
        Am[i, j] -= h
        fd = (loss(Ap) - loss(Am)) / (2 * h)
        assert fd == pytest.approx(gA[i, j], rel=1e-5, abs=1e-7)
    # and grad_b is the gradient with respect to b
    for _ in range(6):
        i, r = rng.integers(0, n), rng.integers(0, nrhs)
        Bp, Bm = B.copy(), B.copy()
        Bp[i, r] += h
        Bm[i, r] -= h
        fp = orc.factor(A, orc.TOEPLITZ, 5)
        lp = float(np.sum(Wt * orc.solve(fp, Bp, refine=2).X))
        lm = float(np.sum(Wt * orc.solve(fp, Bm, refine=2).X))
        assert (lp - lm) / (2 * h) == pytest.approx(gb[i, r], rel=1e-6, abs=1e-8)


def test_refinement_reduces_backward_error(orc):
    A = workloads.conditioned(128, 1e8, seed=4)
    b = workloads.rhs(128, 2, seed=4)
    f = orc.factor(A, orc.GAUSSIAN, 3)
    s = orc.solve(f, b, refine=3)
    assert s.eta[1] <= s.eta[0]
    assert s.eta[-1] <= 1e-15


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
@pytest.mark.parametrize("block", [8, 40, 200])
def test_local_pivot_solve_and_adjoint_match_lapack(orc, kind, block):
    # P A H = L U: x = H U^{-1} L^{-1} P b and A^{-T} w = P^T L^{-T} U^{-T} H^T w
    n = 150
    A = workloads.conditioned(n, 1e4, seed=9)
    B = workloads.rhs(n, 2, seed=9)
    W = workloads.rhs(n, 3, seed=10)
    f = orc.factor(A, kind, seed=12, pivot_blocks=library_blocks(n, block))
    assert f.status == orc.OK
    s = orc.solve(f, B, refine=1)
    X = np.linalg.solve(A, B)
    assert np.linalg.norm(s.X - X) / np.linalg.norm(X) <= 8 * 1e4 * n * EPS
    assert s.eta[-1] <= 1e-15
    Y = orc.solve_adjoint(f, W)
    want = np.linalg.solve(A.T, W)
    np.testing.assert_allclose(Y, want, rtol=0, atol=1e-10 * np.abs(want).max())


@pytest.mark.parametrize("seed", range(2))
def test_breakdown_case_local_pivot(orc, seed):
    # the leading 64 x 64 block is singular: windows of 64 meet an exact zero at
    # 63 without a multiplier; windows of 128 pivot past it; a Gaussian
    # multiplier makes every window's leading block nonsingular
    A = workloads.breakdown_case(seed)
    b = workloads.rhs(256, 1, seed)
    f = orc.factor(A, orc.NONE, 0, pivot_blocks=library_blocks(256, 64))
    assert f.status == orc.ZERO_PIVOT and f.info == 63
    f = orc.factor(A, orc.NONE, 0, pivot_blocks=library_blocks(256, 128))
    assert f.status == orc.OK
    f = orc.factor(A, orc.GAUSSIAN, seed + 1000, pivot_blocks=library_blocks(256, 64))
    assert f.status == orc.OK
    assert orc.solve(f, b, refine=1).eta[-1] <= 1e-15
