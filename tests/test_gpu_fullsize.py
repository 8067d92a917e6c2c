"""Full-size checks in the launch configuration bench.py times, plus the n = 4096 and
n = 8192 workloads, through the C ABI.

At n = 16384 the oracle cannot factor the matrix in a test's time, so the checks are
* sampled entries the oracle computes one by one: entries of M = A G against the oracle's
  multiplier (|M_g - M_o| <= 2 (n + 4) u (|A| |G|)), and entries of L U - P M against the
  blocked-elimination backward bound 8 n u k32 (|L| |U|) of the unpivoted tests;
* properties that hold at any size: the normwise backward error eta of the returned x,
  recomputed here on the host in FP64, is <= 1e-14.
At n = 4096 (Gaussian and circulant multipliers, kappa 1e2 / 1e6 / 1e10, 8 right-hand sides)
the solutions are compared with the oracle's element by element; at n = 8192 (Toeplitz
multiplier, 16 right-hand sides) with LAPACK's solution and through the adjoint identity
w . (A^{-1} b) = (A^{-T} w) . b.
"""
import numpy as np
import pytest

import oracle
import workloads
from test_gpu_parity import dev, host

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps
N = 16384
BENCH_SEED = 1  # bench.py's default workload: kappa = precision_kappa(1) = 12.5


@pytest.fixture(scope="module")
def rmge():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1406_5802_amd as m

    m.lib()
    return m


@pytest.fixture(scope="module")
def big():
    """The bench input (A on the GPU and on the host, b) and the oracle's dense G."""
    kappa = workloads.precision_kappa(BENCH_SEED)
    A = workloads.conditioned_torch(N, kappa, BENCH_SEED)
    b = workloads.rhs_torch(N, 1, BENCH_SEED)
    G = oracle.multiplier(oracle.GAUSSIAN, N, BENCH_SEED + 1000)
    return A, host(A), b, host(b), G, kappa


def _eta(Ah, x, b):
    r = b - Ah @ x
    return np.abs(r).max() / (np.abs(Ah).sum(axis=1).max() * np.abs(x).max() + np.abs(b).max())


def _sample(n, count, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, n, count), rng.integers(0, n, count)


def test_fullsize_product_sampled(rmge, big):
    A, Ah, _, _, G, _ = big
    M = host(rmge.precondition(A, rmge.GAUSSIAN, BENCH_SEED + 1000))
    ii, jj = _sample(N, 2000, 1)
    want = np.einsum("ij,ji->i", Ah[ii], G[:, jj])
    bound = 2 * (N + 4) * EPS * np.einsum("ij,ji->i", np.abs(Ah[ii]), np.abs(G[:, jj]))
    err = np.abs(M[ii, jj] - want)
    assert (err <= bound).all(), float((err / bound).max())


def _k32(LU, n):
    k = 1.0
    for s in range(0, n, 32):
        e = min(n, s + 32)
        Lb = np.tril(LU[s:e, s:e], -1) + np.eye(e - s)
        Ub = np.triu(LU[s:e, s:e])
        k = max(k, np.linalg.cond(Lb), np.linalg.cond(Ub))
    return k


@pytest.mark.parametrize("prec,pivot", [("F64", "PIVOT_NONE"), ("F32", "PIVOT_BLOCK"),
                                        ("F32_BF16X2", "PIVOT_BLOCK")])
def test_fullsize_factors_sampled(rmge, big, prec, pivot):
    A, Ah, _, _, G, _ = big
    split = prec == "F32_BF16X2"
    if split:  # the split path's multiplier is the draw rounded to BF16
        from test_gpu_split16 import _bf16

        G = _bf16(G)
    f = rmge.factor(A, kind=rmge.GAUSSIAN, seed=BENCH_SEED + 1000, block=256,
                    prec=getattr(rmge, prec), pivot=getattr(rmge, pivot))
    assert f.ok, f.status
    LU = host(f.lu())
    perm = host(f.perm()).astype(np.int64)
    for s in range(0, N, 128):  # rows never leave their 128-row block
        assert sorted(perm[s:s + 128]) == list(range(s, min(N, s + 128)))
    ii, jj = _sample(N, 400, 2)
    u = EPS if prec == "F64" else np.finfo(np.float32).eps / 2
    k32 = _k32(LU, N)
    for i, j in zip(ii, jj):
        m = min(i, j)
        # (L U)_ij = sum_{k <= min(i, j)} L_ik U_kj with L_ii = 1
        k = np.arange(m + 1)
        Lrow = np.where(k < i, LU[i, :m + 1], np.where(k == i, 1.0, 0.0))
        Ucol = np.where(k <= j, LU[:m + 1, j], 0.0)
        lu_ij = float(Lrow @ Ucol)
        m_ij = float(Ah[perm[i]] @ G[:, j])
        # FP32: M itself is the FP32 product of A rounded to FP32 and G rounded to FP32;
        # split: A in two BF16 terms (2^-17 relative left out) times the BF16 G
        mbound = (2 * (N + 4) * u + (2.0 ** -17 if split else 0.0)) * float(
            np.abs(Ah[perm[i]]) @ np.abs(G[:, j]))
        bound = 8 * N * u * k32 * float(np.abs(Lrow) @ np.abs(Ucol)) + mbound
        assert abs(lu_ij - m_ij) <= bound, (i, j, lu_ij, m_ij, bound)


# the bench's paths: (multiplier, factor precision, row exchanges, refinement)
FULL_PATHS = {"f64": ("GAUSSIAN", "F64", "PIVOT_NONE", "ir"),
              "f32pg": ("GAUSSIAN", "F32", "PIVOT_BLOCK", "gmres"),
              "f32xpg": ("GAUSSIAN", "F32_BF16X2", "PIVOT_BLOCK", "gmres"),
              "u64": ("UNITARY_CIRCULANT", "F64", "PIVOT_NONE", "ir"),
              "u32xg": ("UNITARY_CIRCULANT", "F32_BF16X2", "PIVOT_NONE", "gmres")}


@pytest.mark.parametrize("path", sorted(FULL_PATHS))
def test_fullsize_solve_backward_error(rmge, big, path):
    A, Ah, b, bh, _, _ = big
    kind, prec, pivot, method = FULL_PATHS[path]
    f = rmge.factor(A, kind=getattr(rmge, kind), seed=BENCH_SEED + 1000, block=256,
                    prec=getattr(rmge, prec), pivot=getattr(rmge, pivot))
    assert f.ok, f.status
    if method == "ir":
        X, st = f.solve(b, max_refine=16, tol=1e-14)
    else:
        X, st = f.solve_gmres(b, max_iters=200, restart=32, tol=1e-14)
    assert st["converged"], st
    eta = _eta(Ah, host(X)[:, 0], bh[:, 0])
    assert eta <= 1e-14, (eta, st["eta"])
    assert eta == pytest.approx(st["eta"], rel=0.5, abs=1e-15)


@pytest.mark.parametrize("kind,n", [("CIRCULANT", 16384), ("UNITARY_CIRCULANT", 16384),
                                    ("TOEPLITZ", 8192), ("CIRCULANT", 5000)])
def test_fullsize_fft_product_rows(rmge, kind, n):
    # the FFT launch at its largest period, m = 16384 (n = 16384 circulants;
    # n = 8192 Toeplitz and n = 5000 circulant embedded in m = 16384), sampled
    # rows against the oracle's plain product with its dense multiplier:
    # |M_g - M_o| <= 16 u log2(m) ||a_i|| ||h|| per row (sqrt 2 more when embedded)
    import math

    k = getattr(rmge, kind)
    A = workloads.gaussian_torch(n, seed=n)
    M = rmge.precondition(A, k, seed=55)
    rows = np.random.default_rng(n).integers(0, n, 12)
    Ah = host(A[rows])
    Mg = host(M[rows])
    H = oracle.multiplier(k, n, 55)
    Mo = oracle.matmul(Ah, H)
    del H
    circ = kind != "TOEPLITZ"
    m = 16384
    hnorm = np.linalg.norm(oracle.multiplier_params(k, n, 55))
    if not (circ and n == m):
        hnorm *= math.sqrt(2)
    bound = 16 * EPS * math.log2(m) * np.linalg.norm(Ah, axis=1) * hnorm
    err = np.abs(Mg - Mo).max(axis=1)
    assert (err <= bound).all(), float((err / bound).max())


@pytest.fixture(scope="module")
def mid_inputs():
    cache = {}

    def get(kappa):
        if kappa not in cache:
            cache[kappa] = workloads.conditioned(4096, kappa, seed=int(np.log10(kappa)))
        return cache[kappa]
    return get


@pytest.mark.parametrize("kappa", [1e2, 1e6, 1e10])
@pytest.mark.parametrize("kind", ["GAUSSIAN", "CIRCULANT"])
def test_n4096_block256_matches_oracle(rmge, mid_inputs, kind, kappa):
    n = 4096
    A = mid_inputs(kappa)
    B = workloads.rhs(n, 8, seed=7)
    k = getattr(rmge, kind)
    f = rmge.factor(dev(A), kind=k, seed=77, block=256)
    assert f.ok
    X, st = f.solve(dev(B), max_refine=1)
    fo = oracle.factor(A, k, 77)
    so = oracle.solve(fo, B, refine=1)
    rel = np.linalg.norm(host(X) - so.X) / np.linalg.norm(so.X)
    assert rel <= max(1e-10, 2 * kappa * (st["eta"] + so.eta[-1])), (rel, st["eta"], so.eta[-1])
    # one classical step reaches what the method reaches in FP64 (the oracle's eta); at
    # kappa = 1e10, kappa(A G) u times the growth is near 1 and neither side gets to 1e-13
    assert st["eta"] <= max(1e-13, 10 * so.eta[-1]), (st["eta"], so.eta)
    # GMRES-based refinement with the same factors reaches 1e-14 across the range
    X2, st2 = f.solve_gmres(dev(B), max_iters=300, restart=32, tol=1e-14)
    assert st2["converged"], st2
    rel = np.linalg.norm(host(X2) - so.X) / np.linalg.norm(so.X)
    assert rel <= max(1e-10, 2 * kappa * (st2["eta"] + so.eta[-1])), rel


@pytest.mark.parametrize("prec", ["F64", "F32"])
def test_n8192_toeplitz_16rhs(rmge, prec):
    n, kappa = 8192, 1e3
    A = workloads.conditioned_torch(n, kappa, seed=4)
    Ah = host(A)
    B = workloads.rhs_torch(n, 16, seed=4)
    W = workloads.rhs_torch(n, 16, seed=5)
    f = rmge.factor(A, kind=rmge.TOEPLITZ, seed=9, block=256, prec=getattr(rmge, prec),
                    pivot=rmge.PIVOT_BLOCK if prec == "F32" else rmge.PIVOT_NONE)
    assert f.ok
    if prec == "F64":
        X, st = f.solve(B, max_refine=4, tol=1e-14)
    else:
        X, st = f.solve_gmres(B, max_iters=400, restart=32, tol=1e-14)
    assert st["converged"], st
    Xh = host(X)
    Xl = np.linalg.solve(Ah, host(B))
    rel = np.linalg.norm(Xh - Xl) / np.linalg.norm(Xl)
    assert rel <= max(1e-10, 4 * kappa * (st["eta"] + n * EPS)), rel
    if prec == "F64":
        Y, sta = f.solve_adjoint_refined(W, max_refine=16, tol=1e-14)
    else:
        Y, sta = f.solve_gmres(W, max_iters=400, restart=32, tol=1e-14, trans=True)
    assert sta["converged"], sta
    Y = host(Y)
    lhs = np.einsum("ir,ir->r", host(W), Xh)
    rhs = np.einsum("ir,ir->r", Y, host(B))
    assert np.allclose(lhs, rhs, rtol=1e-9 * kappa, atol=0), (lhs[:3], rhs[:3])
