"""GPU path vs the FP64 oracle for block elimination with partial pivoting
inside the small diagonal blocks (Section 3, after eq. eqgenpin: the recursion
of eq. eqgenp stops at small blocks handled by a black-box method).

The row order is an integer result decided by floating-point comparisons; the
GPU and the oracle both compare FP64 magnitudes, and on these seeded inputs no
two candidates are within rounding of each other, so the permutations must be
identical.  Tolerances for the factors and solutions are those of the
unpivoted tests (derived there from the arithmetic), applied to P M.
"""
import numpy as np
import pytest

import oracle
import workloads
from partition import library_blocks
from test_gpu_parity import _kappa32, _kappa_leading, dev, host

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def rmge():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1406_5802_amd as m

    m.lib()
    return m


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
@pytest.mark.parametrize("n,block", [(64, 64), (129, 32), (300, 256), (300, 100), (517, 256),
                                     (517, 128), (200, 7), (96, 1), (45, 2), (260, 130)])
def test_pivoted_factors_match_oracle(rmge, kind, n, block):
    A = workloads.conditioned(n, 1e2, seed=31)
    f = rmge.factor(dev(A), kind=kind, seed=17, block=block, pivot=rmge.PIVOT_BLOCK)
    assert f.ok, f.status
    fo = oracle.factor(A, kind, 17, pivot_blocks=library_blocks(A.shape[0], block))
    assert fo.status == oracle.OK
    perm = host(f.perm()).astype(np.int64)
    np.testing.assert_array_equal(perm, fo.perm)
    LU = host(f.lu())
    Mo = oracle.matmul(A, fo.H)
    PM = Mo[fo.perm]
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    back = np.abs(L @ U - PM).max()
    mdiff = 2 * (n + 4) * EPS * (np.abs(A) @ np.abs(fo.H)).max()
    bound = 8 * n * EPS * _kappa32(L, U) * (np.abs(L) @ np.abs(U)).max() + mdiff
    assert back <= bound, (back, bound)
    growth = max(1.0, np.abs(np.triu(fo.LU)).max() / np.abs(Mo).max())
    rel = np.abs(LU - fo.LU).max() / np.abs(fo.LU).max()
    fwd = 8 * n * EPS * _kappa_leading(PM) * growth
    assert rel <= fwd, (rel, fwd)


def test_unpivoted_handle_reports_identity(rmge):
    A = workloads.conditioned(40, 10.0, seed=2)
    f = rmge.factor(dev(A), kind=rmge.GAUSSIAN, seed=3, block=16)
    np.testing.assert_array_equal(host(f.perm()), np.arange(40))


@pytest.mark.parametrize("block", [1, 32, 64])
def test_pivoted_breakdown_on_singular_boundary_block(rmge, block):
    # A[63, 0:64] = 0: the leading 64 x 64 block is singular.  Blocks ending at
    # 64 meet an exact zero at 63; pivoting cannot move row 63 out of its block.
    A = workloads.breakdown_case(seed=0)
    f = rmge.factor(dev(A), kind=rmge.NONE, seed=0, block=block, pivot=rmge.PIVOT_BLOCK)
    assert f.status == 4 and f.info == 63
    fo = oracle.factor(A, oracle.NONE, 0, pivot_blocks=library_blocks(A.shape[0], block))
    assert fo.status == oracle.ZERO_PIVOT and fo.info == 63


@pytest.mark.parametrize("block", [100, 128, 256])
def test_pivoted_elimination_passes_singular_inner_block(rmge, block):
    # no block boundary at 64: the singular leading 64 block is not a pivot block
    A = workloads.breakdown_case(seed=1)
    b = workloads.rhs(256, 1, 1)
    f = rmge.factor(dev(A), kind=rmge.NONE, seed=0, block=block, pivot=rmge.PIVOT_BLOCK)
    assert f.ok, f.status
    X, st = f.solve(dev(b), max_refine=1)
    assert st["eta"] <= 1e-13, st
    fo = oracle.factor(A, oracle.NONE, 0, pivot_blocks=library_blocks(A.shape[0], block))
    so = oracle.solve(fo, b, refine=1)
    kappa = np.linalg.cond(A)
    rel = np.linalg.norm(host(X) - so.X) / np.linalg.norm(so.X)
    assert rel <= max(1e-10, 2 * kappa * (st["eta"] + so.eta[-1])), rel


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
@pytest.mark.parametrize("n,nrhs,kappa,block", [(70, 1, 1e2, 64), (300, 3, 1e6, 256),
                                                (517, 8, 1e2, 128), (129, 17, 1e4, 32)])
def test_pivoted_solve_and_adjoint_match_oracle(rmge, kind, n, nrhs, kappa, block):
    A = workloads.conditioned(n, kappa, seed=41)
    B = workloads.rhs(n, nrhs, seed=42)
    W = workloads.rhs(n, nrhs, seed=43)
    f = rmge.factor(dev(A), kind=kind, seed=23, block=block, pivot=rmge.PIVOT_BLOCK)
    assert f.ok
    X, st = f.solve(dev(B), max_refine=1)
    assert st["eta"] <= 1e-13, st
    fo = oracle.factor(A, kind, 23, pivot_blocks=library_blocks(A.shape[0], block))
    so = oracle.solve(fo, B, refine=1)
    rel = np.linalg.norm(host(X) - so.X) / np.linalg.norm(so.X)
    assert rel <= max(1e-10, 2 * kappa * (st["eta"] + so.eta[-1])), rel
    Y = host(f.solve_adjoint(dev(W)))
    Yo = oracle.solve_adjoint(fo, W)
    rel = np.linalg.norm(Y - Yo) / np.linalg.norm(Yo)
    assert rel <= max(1e-9, 8 * kappa * n * EPS), rel


@pytest.mark.parametrize("kind", [1, 2])
@pytest.mark.parametrize("n,kappa", [(384, 1e2), (1000, 1e2)])
def test_pivoted_fp32_refined_to_fp64(rmge, kind, n, kappa):
    # classical refinement contracts by about kappa(A H) u_32 per step, so it
    # needs kappa(A) kappa(H) well below 1 / u_32
    A = workloads.conditioned(n, kappa, seed=12)
    B = workloads.rhs(n, 2, seed=13)
    f = rmge.factor(dev(A), kind=kind, seed=5, block=256, prec=rmge.F32, pivot=rmge.PIVOT_BLOCK)
    assert f.ok
    X, st = f.solve(dev(B), max_refine=16, tol=1e-14)
    assert st["converged"] and st["eta"] <= 1e-14, st
    fo = oracle.factor(A, kind, 5, pivot_blocks=library_blocks(A.shape[0], 256))
    so = oracle.solve(fo, B, refine=1)
    rel = np.linalg.norm(host(X) - so.X) / np.linalg.norm(so.X)
    assert rel <= max(1e-10, 2 * kappa * (st["eta"] + so.eta[-1])), rel


def test_pivoted_block_sizes_agree_on_the_solution(rmge):
    n = 300
    A = workloads.conditioned(n, 1e3, seed=14)
    b = workloads.rhs(n, 1, seed=15)
    fo = oracle.factor(A, oracle.GAUSSIAN, 9, pivot_blocks=library_blocks(A.shape[0], 64))
    xo = oracle.solve(fo, b, refine=1).X
    for block in (1, 2, 3, 7, 32, 64, 128, 200, 256):
        f = rmge.factor(dev(A), kind=rmge.GAUSSIAN, seed=9, block=block, pivot=rmge.PIVOT_BLOCK)
        X, st = f.solve(dev(b), max_refine=1)
        rel = np.linalg.norm(host(X) - xo) / np.linalg.norm(xo)
        assert rel <= 1e-10, (block, rel)
