"""GMRES-based refinement (rmge_solve_gmres) against the FP64 oracle.

The refined solution is the unique solution of A x = b, so it is compared with
the oracle's (GENP plus one classical refinement step in FP64) by the solution
tolerance of the other parity tests: ||x_g - x_o|| / ||x_o|| <= max(1e-10,
2 kappa (eta_g + eta_o)); eta_g <= 1e-14 is required of every converged run.
"""
import numpy as np
import pytest

import oracle
import workloads
from test_gpu_parity import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rmge():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1406_5802_amd as m

    m.lib()
    return m


def _check(X, A, B, kind, seed, kappa, eta):
    fo = oracle.factor(A, kind, seed)
    so = oracle.solve(fo, B, refine=1)
    rel = np.linalg.norm(host(X) - so.X) / np.linalg.norm(so.X)
    assert rel <= max(1e-10, 2 * kappa * (eta + so.eta[-1])), rel


@pytest.mark.parametrize("kind", [1, 2, 3])
@pytest.mark.parametrize("prec", ["F64", "F32"])
@pytest.mark.parametrize("pivot", ["PIVOT_NONE", "PIVOT_BLOCK"])
def test_gmres_matches_oracle(rmge, kind, prec, pivot):
    n, nrhs, kappa = 300, 2, 1e4
    A = workloads.conditioned(n, kappa, seed=51)
    B = workloads.rhs(n, nrhs, seed=52)
    f = rmge.factor(dev(A), kind=kind, seed=29, block=128, prec=getattr(rmge, prec),
                    pivot=getattr(rmge, pivot))
    assert f.ok
    X, st = f.solve_gmres(dev(B), max_iters=200, restart=32, tol=1e-14)
    assert st["converged"] and st["eta"] <= 1e-14, st
    _check(X, A, B, kind, 29, kappa, st["eta"])


@pytest.mark.parametrize("pivot", ["PIVOT_BLOCK"])
def test_gmres_converges_where_classical_refinement_stalls(rmge, pivot):
    # FP32 factors of A G with kappa(A) = 1e6 at n = 1000: kappa(A G) u_32 >> 1,
    # so classical refinement cannot contract; the Krylov iteration still can,
    # given factors with small growth (pivoting inside the diagonal blocks; the
    # unpivoted FP32 factors of this input, growth ~1e3, stall restarted GMRES
    # as well).
    n, kappa = 1000, 1e6
    A = workloads.conditioned(n, kappa, seed=61)
    b = workloads.rhs(n, 1, seed=62)
    f = rmge.factor(dev(A), kind=rmge.GAUSSIAN, seed=33, block=256, prec=rmge.F32,
                    pivot=getattr(rmge, pivot))
    assert f.ok
    _, st_ir = f.solve(dev(b), max_refine=16, tol=1e-14)
    X, st = f.solve_gmres(dev(b), max_iters=400, restart=64, tol=1e-14)
    assert st["converged"] and st["eta"] <= 1e-14, (st, st_ir["eta_hist"])
    _check(X, A, b, rmge.GAUSSIAN, 33, kappa, st["eta"])


def test_gmres_iteration_cap_and_restart(rmge):
    n, kappa = 500, 1e5
    A = workloads.conditioned(n, kappa, seed=71)
    b = workloads.rhs(n, 1, seed=72)
    f = rmge.factor(dev(A), kind=rmge.CIRCULANT, seed=5, block=64, prec=rmge.F32)
    X0, st0 = f.solve_gmres(dev(b), max_iters=0, restart=8, tol=1e-14)
    assert st0["iters"] == 0 and not st0["converged"]
    X, st = f.solve_gmres(dev(b), max_iters=300, restart=4, tol=1e-14)  # many restarts
    assert st["converged"] and st["eta"] <= 1e-14, st
    assert st["iters"] <= 300
    _check(X, A, b, rmge.CIRCULANT, 5, kappa, st["eta"])


@pytest.mark.parametrize("kind", [1, 2, 3])
@pytest.mark.parametrize("prec", ["F64", "F32"])
def test_gmres_adjoint_matches_oracle(rmge, kind, prec):
    n, nrhs, kappa = 300, 2, 1e4
    A = workloads.conditioned(n, kappa, seed=81)
    W = workloads.rhs(n, nrhs, seed=82)
    f = rmge.factor(dev(A), kind=kind, seed=6, block=128, prec=getattr(rmge, prec),
                    pivot=rmge.PIVOT_BLOCK)
    Y, st = f.solve_gmres(dev(W), max_iters=200, restart=32, tol=1e-14, trans=True)
    assert st["converged"] and st["eta"] <= 1e-14, st
    Yo = np.linalg.solve(A.T, W)
    rel = np.linalg.norm(host(Y) - Yo) / np.linalg.norm(Yo)
    assert rel <= max(1e-10, 4 * kappa * n * np.finfo(float).eps), rel


@pytest.mark.parametrize("kind,trans,nrhs", [(1, False, 17), (2, False, 16), (3, True, 5)])
def test_gmres_block_matches_columns_alone(rmge, kind, trans, nrhs):
    # several right-hand sides advance their Arnoldi processes together
    # (one preconditioner application and one product with op(A) for all of
    # them): each column must reach what the same refinement reaches for it
    # alone, and the backward error recomputed here must meet the tolerance
    import torch

    n, kappa = 400, 1e3
    A = workloads.conditioned(n, kappa, seed=91)
    B = workloads.rhs(n, nrhs, seed=92)
    f = rmge.factor(dev(A), kind=kind, seed=7, block=128, prec=rmge.F32, pivot=rmge.PIVOT_BLOCK)
    assert f.ok
    X, st = f.solve_gmres(dev(B), max_iters=300, restart=32, tol=1e-14, trans=trans)
    assert st["converged"] and st["eta"] <= 1e-14, st
    Xh = host(X)
    Aop = A.T if trans else A
    anorm = np.abs(Aop).sum(axis=1).max()
    for c in range(nrhs):
        x1, st1 = f.solve_gmres(dev(np.ascontiguousarray(B[:, c:c + 1])), max_iters=300,
                                restart=32, tol=1e-14, trans=trans)
        assert st1["converged"]
        x = Xh[:, c]
        r = B[:, c] - Aop @ x
        eta = np.abs(r).max() / (anorm * np.abs(x).max() + np.abs(B[:, c]).max())
        assert eta <= 1e-14, (c, eta)
        rel = np.linalg.norm(x - host(x1)[:, 0]) / np.linalg.norm(host(x1))
        assert rel <= max(1e-10, 2 * kappa * (eta + st1["eta"])), (c, rel)
    torch.cuda.synchronize()
