"""Batches of uneven systems (rmge_batch_*) against the oracle, through the C ABI.

Each system is the single-system method with FP32 factors: its multiplier from
its own seed (dense Gaussian, or circulant with a Gaussian first column),
M = A H, GENP in FP32 with pivot blocks of nb columns, FP64 GMRES refinement.
Tolerances (as for the single-system FP32 tests):
* solutions: ||x_g - x_o|| / ||x_o|| <= max(1e-10, 2 kappa (eta_g + eta_o)), the
  oracle's x after one FP64 refinement step; eta_g recomputed here <= 1e-14;
* factors: ||L U - M||_max <= 8 n u32 || |L| |U| ||_max + (product error), M the
  oracle's product with A (and a Gaussian G) rounded to FP32 (blocked
  elimination whose block solves are substitutions is backward stable, Higham,
  Accuracy and Stability, Thm 9.3 / 13.x);
* a system whose FP32 stage stalls is solved again from FP64 factors, and says so;
* a zero leading block gives RMGE_ZERO_PIVOT at index 0 for its system only;
* a run replayed from the HIP graph gives the eager run's results bit for bit.
"""
import numpy as np
import pytest

import oracle
import workloads
from test_gpu_parity import host

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24
EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def rmge():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1406_5802_amd as m

    m.lib()
    return m


SIZES = [1, 2, 3, 7, 16, 31, 33, 64, 65, 100, 127, 128, 129, 200, 256, 257, 300, 511, 513, 700]


def _make(sizes, kappas, seed0=0):
    """Host matrices, right-hand sides and the system table (offsets into flat buffers)."""
    systems, As, bs = [], [], []
    a_off = v_off = 0
    for i, (n, kappa) in enumerate(zip(sizes, kappas)):
        kind = 1 if i % 2 == 0 else 2  # Gaussian, circulant alternately
        A = workloads.conditioned(n, kappa, seed=seed0 + i) if n > 1 else np.array([[0.7]])
        b = workloads.rhs(n, 1, seed=seed0 + 500 + i)[:, 0]
        systems.append((n, kind, 9000 + i, a_off, v_off))
        As.append(A)
        bs.append(b)
        a_off += n * n
        v_off += n
    return systems, As, bs


def _flat(rmge, As, bs):
    import torch

    A = torch.as_tensor(np.concatenate([a.ravel() for a in As]), device="cuda")
    B = torch.as_tensor(np.concatenate(bs), device="cuda")
    X = torch.full_like(B, float("nan"))
    return A, B, X


def _eta(A, x, b):
    r = b - A @ x
    return np.abs(r).max() / (np.abs(A).sum(axis=1).max() * np.abs(x).max() + np.abs(b).max())


def _check_solutions(systems, As, bs, X, res, tol=1e-14):
    for i, ((n, kind, seed, _, vo), A, b) in enumerate(zip(systems, As, bs)):
        assert res["status"][i] == 0, (i, n, kind, res["status"][i], res["eta"][i])
        x = X[vo:vo + n]
        eta = _eta(A, x, b)
        assert eta <= tol, (i, n, kind, eta)
        assert eta == pytest.approx(res["eta"][i], rel=0.5, abs=1e-16)
        fo = oracle.factor(A, kind, seed)
        so = oracle.solve(fo, b[:, None], refine=1)
        kappa = np.linalg.cond(A)
        rel = np.linalg.norm(x - so.X[:, 0]) / np.linalg.norm(so.X[:, 0])
        assert rel <= max(1e-10, 2 * kappa * (eta + so.eta[-1])), (i, n, kind, rel)


def test_batch_matches_oracle(rmge):
    kappas = [1e2 if i % 3 else 1e4 for i in range(len(SIZES))]
    systems, As, bs = _make(SIZES, kappas)
    A, B, X = _flat(rmge, As, bs)
    bt = rmge.Batch(systems, restart=16, max_iters=300)
    bt.run(A, B, X, tol=1e-14)
    res = bt.results()
    _check_solutions(systems, As, bs, host(X), res)
    assert (res["info"] == -1).all()
    assert (res["eta0"] >= res["eta"]).all()


@pytest.mark.parametrize("tuning", [[16, 16, 16, 16, 16], [32, 32, 32, 32, 32], [64, 64, 64, 64, 64]])
def test_batch_factors_match_oracle(rmge, tuning):
    sizes = [33, 100, 129, 300, 520]
    systems, As, bs = _make(sizes, [1e2] * len(sizes), seed0=40)
    A, B, X = _flat(rmge, As, bs)
    bt = rmge.Batch(systems, tuning=tuning, restart=16, max_iters=300)
    bt.run(A, B, X, tol=1e-14)
    res = bt.results()
    _check_solutions(systems, As, bs, host(X), res)
    for i, ((n, kind, seed, _, _), Ah) in enumerate(zip(systems, As)):
        LU = host(bt.lu(i, n))
        L = np.tril(LU, -1) + np.eye(n)
        U = np.triu(LU)
        A32 = Ah.astype(np.float32).astype(np.float64)
        H = oracle.multiplier(kind, n, seed)
        if kind == 1:  # FP32 product of A and G, both rounded to FP32
            H32 = H.astype(np.float32).astype(np.float64)
            Mo = oracle.matmul(A32, H32)
            mdiff = 2 * (n + 4) * U32 * (np.abs(A32) @ np.abs(H32)).max()
        else:  # FFT of the FP64 row, rounded to FP32 once
            Mo = oracle.matmul(Ah, H)
            mdiff = (U32 + 16 * EPS * np.log2(2 * n)) * (np.abs(Ah) @ np.abs(H)).max()
        back = np.abs(L @ U - Mo).max()
        bound = 8 * n * U32 * (np.abs(L) @ np.abs(U)).max() + mdiff
        assert back <= bound, (i, n, kind, back, bound)


def test_batch_breakdown_is_per_system(rmge):
    sizes = [50, 80, 120]
    systems, As, bs = _make(sizes, [1e2] * 3, seed0=70)
    As[1] = np.zeros((80, 80))  # M = 0: the first pivot is zero
    A, B, X = _flat(rmge, As, bs)
    bt = rmge.Batch(systems, restart=16, max_iters=300)
    bt.run(A, B, X, tol=1e-14)
    res = bt.results()
    assert res["status"][1] == 4 and res["info"][1] == 0
    Xh = host(X)
    assert np.isnan(Xh[systems[1][4]:systems[1][4] + 80]).all()  # left untouched
    keep = [0, 2]
    _check_solutions([systems[i] for i in keep], [As[i] for i in keep], [bs[i] for i in keep],
                     Xh, {k: v[keep] for k, v in res.items()})


def test_batch_graph_replays_match_eager(rmge):
    import torch

    sizes = [20, 64, 97, 130, 260, 400]
    systems, As, bs = _make(sizes, [1e3] * len(sizes), seed0=90)
    A, B, X = _flat(rmge, As, bs)
    bt = rmge.Batch(systems, restart=16, max_iters=300)
    bt.run(A, B, X, tol=1e-14)
    ref = host(X).copy()
    ref_res = bt.results()
    for rep in range(3):
        X.fill_(float("nan"))
        torch.cuda.synchronize()
        bt.run(A, B, X, tol=1e-14, graph=True)
        got = host(X)
        res = bt.results()
        np.testing.assert_array_equal(got, ref)
        np.testing.assert_array_equal(res["iters"], ref_res["iters"])
        np.testing.assert_array_equal(res["status"], ref_res["status"])
        # eager work on the device between replays
        (torch.randn(512, 512, device="cuda", dtype=torch.float64) @
         torch.randn(512, 512, device="cuda", dtype=torch.float64)).sum().item()
    _check_solutions(systems, As, bs, got, res)


def test_batch_autotune(rmge):
    sizes = [40, 90, 200, 333, 600, 1024]
    systems, As, bs = _make(sizes, [1e2] * len(sizes), seed0=110)
    A, B, X = _flat(rmge, As, bs)
    bt = rmge.Batch(systems, restart=16, max_iters=300)
    nb, ms = bt.autotune(A)
    assert all(v in (16, 32, 64) for v in nb)
    assert nb == bt.tuning()
    assert all(m > 0 for m in ms)  # every bucket has a system here
    bt.run(A, B, X, tol=1e-14)
    _check_solutions(systems, As, bs, host(X), bt.results())
    bt.set_tuning([16, 64, 32, 16, 64])
    assert bt.tuning() == [16, 64, 32, 16, 64]
    bt.run(A, B, X, tol=1e-14)
    _check_solutions(systems, As, bs, host(X), bt.results())


def test_batch_fp64_fallback(rmge):
    # kappa = 1e6 systems with one GMRES iteration allowed for the FP32 stage:
    # those still above tol are solved again from FP64 factors in the same run
    sizes = [90, 180, 333, 520]
    systems, As, bs = _make(sizes, [1e6] * len(sizes), seed0=130)
    A, B, X = _flat(rmge, As, bs)
    bt = rmge.Batch(systems, restart=16, max_iters=1)
    bt.run(A, B, X, tol=1e-14)
    res = bt.results()
    assert res["fp64"].sum() >= 1
    assert (res["iters"] >= 1).all()
    _check_solutions(systems, As, bs, host(X), res)
    # and through the graph
    X.fill_(float("nan"))
    bt.run(A, B, X, tol=1e-14, graph=True)
    res2 = bt.results()
    np.testing.assert_array_equal(res2["fp64"], res["fp64"])
    _check_solutions(systems, As, bs, host(X), res2)
