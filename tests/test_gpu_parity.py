"""GPU path vs the FP64 oracle, element by element, through the C ABI.

Tolerances (written here, derived from the arithmetic; u = 2^-53):
* multiplier parameters: Box-Muller on both sides from bitwise-equal uniforms;
  host libm and device math differ by ulps, so |g - o| <= 4 ulp of the pair's
  radius sqrt(-2 ln u);
* M = A H, dense: |M_g - M_o| <= 2 n u (|A| |H|) elementwise (two FP64
  products of length n), plus the parameters' ulps;  FFT: per row,
  |M_g - M_o| <= 16 u log2(m) ||a||_2 ||h||_2;
* factors: ||L U - M_o||_max <= 8 n u k32 || |L| |U| ||_max + ||M_g - M_o||_max
  (backward error of blocked elimination, Higham, Accuracy and Stability,
  Thm 9.3 / 13.6, with k32 the largest condition number of the 32 x 32
  diagonal sub-blocks that the solves apply through explicit inverses); the
  factors themselves differ from the oracle's unblocked ones by at most
  8 n u kL g (first-order perturbation of LU: kL = max condition of the
  leading principal blocks of M, g = growth max|U| / max|M|);
* solutions: ||x_g - x_o|| / ||x_o|| <= max(1e-10, 2 kappa (eta_g + eta_o)),
  the 1e-10 bound wherever conditioning allows it; eta_g <= 1e-13 after at
  most one refinement step.
"""
import math

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def rmge():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1406_5802_amd as m

    m.lib()
    return m


def dev(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def _eta(M, X, B):
    """Largest normwise backward error max_j |B_j - M X_j| / (|M| |X_j| + |B_j|), 2-norms."""
    X = X.reshape(X.shape[0], -1)
    B = B.reshape(B.shape[0], -1)
    nm = np.linalg.norm(M, 2)
    r = np.linalg.norm(B - M @ X, axis=0)
    return float(np.max(r / (nm * np.linalg.norm(X, axis=0) + np.linalg.norm(B, axis=0))))


def _pair_radius(z):
    z = np.asarray(z)
    pad = (-z.size) % 4
    zz = np.concatenate([z, np.zeros(pad)]).reshape(-1, 2)
    r = np.sqrt((zz ** 2).sum(axis=1))
    return np.repeat(r, 2)[: z.size]


@pytest.mark.parametrize("kind,n", [(1, 1), (1, 3), (1, 64), (1, 257), (2, 5), (2, 4096),
                                    (3, 7), (3, 8192)])
def test_multiplier_params_match_oracle(rmge, kind, n):
    seed = 1234 + n
    g = host(rmge.multiplier_params(kind, n, seed))
    o = oracle.multiplier_params(kind, n, seed)
    assert g.shape == o.shape
    tol = 4 * EPS * np.maximum(_pair_radius(o), 1.0)
    bad = np.abs(g - o) > tol
    assert not bad.any(), (np.argwhere(bad)[:5], g[bad][:5], o[bad][:5])


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 64, 1000, 4096, 16384])
def test_unitary_column_matches_oracle(rmge, n):
    # c_k = (1/n) sum of n unit-modulus terms, each within a few ulps on both
    # sides (device: real pairs with cospi; oracle: complex sum with cos, sin)
    seed = 4321 + n
    g = host(rmge.multiplier_params(rmge.UNITARY_CIRCULANT, n, seed))
    o = oracle.multiplier_params(oracle.UNITARY_CIRCULANT, n, seed)
    assert g.shape == o.shape == (n,)
    err = np.abs(g - o).max()
    assert err <= 64 * EPS, err


def _check_product(kind, n, A, M, seed):
    H = oracle.multiplier(kind, n, seed)
    Mo = oracle.matmul(A, H)
    if kind in (0, 1):
        bound = 2 * (n + 4) * EPS * (np.abs(A) @ np.abs(H)) + 1e-300
        err = np.abs(M - Mo)
        assert (err <= bound).all(), float((err / bound).max())
    else:
        circ = kind in (2, 4)
        m = n if (circ and n >= 2 and n & (n - 1) == 0) else max(2, 1 << (2 * n - 2).bit_length())
        hnorm = np.linalg.norm(oracle.multiplier_params(kind, n, seed))
        if circ and m != n:
            hnorm *= math.sqrt(2)
        row_bound = 16 * EPS * max(1, math.log2(m)) * np.linalg.norm(A, axis=1) * hnorm
        err = np.abs(M - Mo).max(axis=1)
        assert (err <= row_bound + 1e-300).all(), float((err / row_bound).max())
    return Mo


@pytest.mark.parametrize("kind", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("n", [1, 2, 7, 64, 128, 129, 300, 384, 512, 517])
def test_precondition_matches_oracle(rmge, kind, n):
    # n a multiple of 128 takes the interior (unchecked) product kernel
    A = workloads.conditioned(n, 1e3, seed=n)
    M = host(rmge.precondition(dev(A), kind, seed=77))
    _check_product(kind, n, A, M, 77)


@pytest.mark.parametrize("kind,n", [(3, 1100), (2, 4096), (4, 3000), (2, 700), (3, 4000),
                                    (4, 4096), (4, 16384)])
def test_precondition_multiwave_rows(rmge, kind, n):
    # periods m = 4096 .. 16384: one row spans several waves of a workgroup;
    # 16 sampled rows against the oracle's plain product (the unitary kind at a
    # power of two takes its spectrum in closed form from the phases)
    A = np.random.default_rng(n).standard_normal((n, n)) / np.sqrt(n)
    M = host(rmge.precondition(dev(A), kind, seed=31))
    rows = np.random.default_rng(n + 1).integers(0, n, 16)
    H = oracle.multiplier(kind, n, 31)
    Mo = oracle.matmul(A[rows], H)
    circ = kind in (2, 4)
    m = n if (circ and n & (n - 1) == 0) else 1 << (2 * n - 2).bit_length()
    hnorm = np.linalg.norm(oracle.multiplier_params(kind, n, 31)) * (1 if m == n else math.sqrt(2))
    bound = 16 * EPS * math.log2(m) * np.linalg.norm(A[rows], axis=1) * hnorm
    err = np.abs(M[rows] - Mo).max(axis=1)
    assert (err <= bound).all(), float((err / bound).max())


def _kappa32(L, U):
    n = L.shape[0]
    k = 1.0
    for i in range(0, n, 32):
        e = min(n, i + 32)
        k = max(k, np.linalg.cond(L[i:e, i:e]), np.linalg.cond(U[i:e, i:e]))
    return k


def _kappa_leading(M):
    n = M.shape[0]
    ks = sorted(set([1, n] + list(range(1, n + 1, max(1, n // 32)))))
    return max(np.linalg.cond(M[:k, :k]) for k in ks)


@pytest.mark.parametrize("kind", [1, 2, 3, 4])
@pytest.mark.parametrize("n,block", [(64, 64), (129, 32), (300, 256), (300, 100), (517, 256),
                                     (517, 128), (200, 7), (96, 1), (45, 2), (77, 3), (512, 256),
                                     (384, 128)])
def test_factors_match_oracle(rmge, kind, n, block):
    A = workloads.conditioned(n, 1e2, seed=3)
    f = rmge.factor(dev(A), kind=kind, seed=11, block=block)
    assert f.ok, f.status
    LU = host(f.lu())
    fo = oracle.factor(A, kind, 11)
    assert fo.status == oracle.OK
    Mo = oracle.matmul(A, fo.H)
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    back = np.abs(L @ U - Mo).max()
    mdiff = 2 * (n + 4) * EPS * (np.abs(A) @ np.abs(fo.H)).max()
    bound = 8 * n * EPS * _kappa32(L, U) * (np.abs(L) @ np.abs(U)).max() + mdiff
    assert back <= bound, (back, bound)
    growth = max(1.0, np.abs(np.triu(fo.LU)).max() / np.abs(Mo).max())
    rel = np.abs(LU - fo.LU).max() / np.abs(fo.LU).max()
    fwd = 8 * n * EPS * _kappa_leading(Mo) * growth
    assert rel <= fwd, (rel, fwd)


@pytest.mark.parametrize("block", [1, 32, 63, 64, 100, 128, 256])
def test_breakdown_zero_pivot(rmge, block):
    A = workloads.breakdown_case(seed=0)
    f = rmge.factor(dev(A), kind=rmge.NONE, seed=0, block=block)
    assert f.status == 4  # RMGE_ZERO_PIVOT
    assert f.info == 63
    with pytest.raises(rmge.RMGEError):
        f.solve(dev(workloads.rhs(256, 1, 0)))
    fo = oracle.factor(A, oracle.NONE, 0)
    assert fo.info == 63


def test_nonfinite_pivot(rmge):
    A = workloads.conditioned(100, 10.0, seed=1)
    A[40, 70] = np.nan
    f = rmge.factor(dev(A), kind=rmge.GAUSSIAN, seed=1, block=32)
    assert f.status == 5  # RMGE_NONFINITE
    assert 0 <= f.info < 100


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("block", [64, 256])
def test_breakdown_case_preprocessed(rmge, seed, block):
    A = workloads.breakdown_case(seed)
    b = workloads.rhs(256, 1, seed)
    f = rmge.factor(dev(A), kind=rmge.GAUSSIAN, seed=seed + 1000, block=block)
    assert f.ok
    X, st = f.solve(dev(b), max_refine=1)
    assert min(st["eta_hist"]) <= 1e-13, st
    fo = oracle.factor(A, oracle.GAUSSIAN, seed + 1000)
    so = oracle.solve(fo, b, refine=1)
    kappa = np.linalg.cond(A)
    rel = np.linalg.norm(host(X) - so.X) / np.linalg.norm(so.X)
    assert rel <= max(1e-10, 2 * kappa * (st["eta"] + so.eta[-1])), rel


@pytest.mark.parametrize("kind", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("n,nrhs,kappa", [(70, 1, 1e2), (300, 3, 1e6), (517, 8, 1e2),
                                          (129, 17, 1e4)])
def test_solve_matches_oracle(rmge, kind, n, nrhs, kappa):
    A = workloads.conditioned(n, kappa, seed=5)
    if kind == 0:
        A = A + n * np.eye(n)  # plain GENP: keep it strongly nonsingular
        kappa = np.linalg.cond(A)
    B = workloads.rhs(n, nrhs, seed=6)
    f = rmge.factor(dev(A), kind=kind, seed=21, block=64)
    assert f.ok
    X, st = f.solve(dev(B), max_refine=1)
    assert st["eta"] <= 1e-13, st
    fo = oracle.factor(A, kind, 21)
    so = oracle.solve(fo, B, refine=1)
    rel = np.linalg.norm(host(X) - so.X) / np.linalg.norm(so.X)
    assert rel <= max(1e-10, 2 * kappa * (st["eta"] + so.eta[-1])), rel


@pytest.mark.parametrize("kind", [0, 1, 2, 3, 4])
def test_adjoint_matches_oracle(rmge, kind):
    n, nrhs = 300, 5
    A = workloads.conditioned(n, 1e3, seed=8)
    if kind == 0:
        A = A + n * np.eye(n)
    W = workloads.rhs(n, nrhs, seed=9)
    f = rmge.factor(dev(A), kind=kind, seed=4, block=128)
    Y = host(f.solve_adjoint(dev(W)))
    fo = oracle.factor(A, kind, 4)
    Yo = oracle.solve_adjoint(fo, W)
    rel = np.linalg.norm(Y - Yo) / np.linalg.norm(Yo)
    # neither side refines: each solution's normwise backward error eta for
    # A^T y = w bounds its forward error by 2 kappa eta (first order), so the
    # two differ by at most 2 kappa (eta_g + eta_o), the rule of the header
    kappa = np.linalg.cond(A)
    bound = 2 * kappa * (_eta(A.T, Y, W) + _eta(A.T, Yo, W))
    assert rel <= max(1e-10, bound), (rel, bound)


@pytest.mark.parametrize("kind", [1, 2, 4])
def test_fp32_factors_refined_to_fp64(rmge, kind):
    n = 384
    A = workloads.conditioned(n, 1e2, seed=12)
    B = workloads.rhs(n, 2, seed=13)
    f = rmge.factor(dev(A), kind=kind, seed=5, block=128, prec=rmge.F32)
    assert f.ok
    X, st = f.solve(dev(B), max_refine=16, tol=1e-14)
    assert st["converged"] and st["eta"] <= 1e-14, st
    fo = oracle.factor(A, kind, 5)
    so = oracle.solve(fo, B, refine=1)
    rel = np.linalg.norm(host(X) - so.X) / np.linalg.norm(so.X)
    assert rel <= 1e-10, rel


def test_block_size_invariance(rmge):
    n = 300
    A = workloads.conditioned(n, 1e3, seed=14)
    b = workloads.rhs(n, 1, seed=15)
    fo = oracle.factor(A, oracle.GAUSSIAN, 9)
    xo = oracle.solve(fo, b, refine=1).X
    for block in (1, 2, 3, 7, 32, 64, 128, 200, 256):
        f = rmge.factor(dev(A), kind=rmge.GAUSSIAN, seed=9, block=block)
        X, st = f.solve(dev(b), max_refine=1)
        rel = np.linalg.norm(host(X) - xo) / np.linalg.norm(xo)
        assert rel <= 1e-10, (block, rel)


@pytest.mark.parametrize("kind", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("prec", ["F64", "F32"])
def test_adjoint_refined_matches_oracle(rmge, kind, prec):
    n, nrhs, kappa = 300, 3, 1e3
    A = workloads.conditioned(n, kappa, seed=18)
    if kind == 0:
        A = A + n * np.eye(n)
        kappa = np.linalg.cond(A)
    W = workloads.rhs(n, nrhs, seed=19)
    f = rmge.factor(dev(A), kind=kind, seed=4, block=128, prec=getattr(rmge, prec))
    Y, st = f.solve_adjoint_refined(dev(W), max_refine=16, tol=1e-14)
    assert st["converged"] and st["eta"] <= 1e-14, st
    Yo = oracle.solve_adjoint(oracle.factor(A, kind, 4), W)
    rel = np.linalg.norm(host(Y) - Yo) / np.linalg.norm(Yo)
    assert rel <= max(1e-10, 4 * kappa * n * EPS), rel
