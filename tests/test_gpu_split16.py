"""FP32 factors with the product M = A H on the BF16 matrix cores
(precision F32_BF16X2): H is the drawn Gaussian rounded to BF16, A is split
into two BF16 terms, and M = A_h H + A_l H accumulates in FP32.

Pins: the factors are checked against the product of A with the BF16-rounded
oracle multiplier (rounding FP64 -> FP32 -> BF16 to nearest even, written out
here with integer arithmetic on the bit patterns), with the FP32 tolerance of
the other factor tests plus the product's own error, |A - A_h - A_l| <= 2^-17 |A|
per term and FP32 accumulation; solutions refined by GMRES against the oracle's
solution (the same x = A^{-1} b whatever the multiplier); other multiplier
kinds give the FP32 factors bit for bit.
"""
import numpy as np
import pytest

import oracle
import workloads
from test_gpu_parity import _kappa32, dev, host

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def rmge():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1406_5802_amd as m

    m.lib()
    return m


def _bf16(x):
    """Round FP64 values to FP32, then to BF16 (nearest, ties to even)."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def test_bf16_rounding_helper():
    # exact cases of the rounding rule: 1 + 2^-8 is a tie (to even: 1), 1 + 3 * 2^-9
    # rounds up to 1 + 2^-7, and BF16 values are fixed points
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, -2.5, 0.0, 3.0 * 2 ** 20])
    want = np.array([1.0, 1.0, 1.0 + 2.0 ** -7, -2.5, 0.0, 3.0 * 2 ** 20])
    np.testing.assert_array_equal(_bf16(x), want)


# Trailing blocks of 2048 rows and more take the three-term BF16 Schur update
# (n = 2300 with 128-column blocks: one step; n = 2600 with 256: two, both
# with ragged 256 x 256 tiles), smaller ones the FP32 kernels.  Blocks of 100
# and 48 columns give update depths that are not whole 32-wide chunks (the
# split zero-fills k up to 128 and 64).
@pytest.mark.parametrize("n,block,pivot", [(256, 128, "PIVOT_BLOCK"), (300, 256, "PIVOT_BLOCK"),
                                           (517, 128, "PIVOT_BLOCK"), (640, 256, "PIVOT_BLOCK"),
                                           (2300, 128, "PIVOT_BLOCK"), (2600, 256, "PIVOT_BLOCK"),
                                           (2300, 256, "PIVOT_NONE"), (2300, 100, "PIVOT_BLOCK"),
                                           (2150, 48, "PIVOT_NONE")])
def test_split16_factors_of_rounded_multiplier(rmge, n, block, pivot):
    A = workloads.conditioned(n, 1e2, seed=31)
    f = rmge.factor(dev(A), kind=rmge.GAUSSIAN, seed=17, block=block, prec=rmge.F32_BF16X2,
                    pivot=getattr(rmge, pivot))
    assert f.ok, f.status
    G = oracle.multiplier(oracle.GAUSSIAN, n, 17)
    Gb = _bf16(G)
    Mb = oracle.matmul(A, Gb)
    perm = host(f.perm()).astype(np.int64)
    LU = host(f.lu())
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    back = np.abs(L @ U - Mb[perm]).max()
    mdiff = (2.0 ** -17 + 2 * (n + 4) * U32) * (np.abs(A) @ np.abs(Gb)).max()
    bound = 8 * n * U32 * _kappa32(L, U) * (np.abs(L) @ np.abs(U)).max() + mdiff
    assert back <= bound, (back, bound)


@pytest.mark.parametrize("n,kappa", [(300, 1e2), (512, 1e3), (1000, 1e2), (2600, 1e2)])
def test_split16_gmres_matches_oracle(rmge, n, kappa):
    A = workloads.conditioned(n, kappa, seed=51)
    B = workloads.rhs(n, 2, seed=52)
    f = rmge.factor(dev(A), kind=rmge.GAUSSIAN, seed=29, block=256, prec=rmge.F32_BF16X2,
                    pivot=rmge.PIVOT_BLOCK)
    assert f.ok
    X, st = f.solve_gmres(dev(B), max_iters=200, restart=32, tol=1e-14)
    assert st["converged"] and st["eta"] <= 1e-14, st
    fo = oracle.factor(A, oracle.GAUSSIAN, 29)
    so = oracle.solve(fo, B, refine=1)
    rel = np.linalg.norm(host(X) - so.X) / np.linalg.norm(so.X)
    assert rel <= max(1e-10, 2 * kappa * (st["eta"] + so.eta[-1])), rel


@pytest.mark.parametrize("kind", ["CIRCULANT", "TOEPLITZ"])
def test_split16_other_kinds_are_fp32(rmge, kind):
    n = 300
    A = dev(workloads.conditioned(n, 1e2, seed=3))
    k = getattr(rmge, kind)
    f1 = rmge.factor(A, kind=k, seed=4, block=128, prec=rmge.F32)
    f2 = rmge.factor(A, kind=k, seed=4, block=128, prec=rmge.F32_BF16X2)
    np.testing.assert_array_equal(host(f1.lu()), host(f2.lu()))


@pytest.mark.parametrize("n", [300, 517])
def test_split16_both_copies_of_h_apply_the_multiplier(rmge, n):
    # The split path keeps H twice: FP32 values (applied for several right-hand
    # sides at once) and BF16 bits transposed (the product, and one right-hand
    # side).  n = 300 draws both in one pass, n = 517 (not a multiple of 4)
    # draws and then rounds.  An unrefined solve x = H U^{-1} L^{-1} b through
    # either copy is as accurate as the FP32 factors allow (~1e-3 here); a copy
    # that is not the multiplier of the factors (misplaced or transposed
    # entries) gives an O(1) error.  (The one- and several-right-hand-side
    # triangular solves round differently, so the two are not compared to
    # each other.)
    A = workloads.conditioned(n, 1e2, seed=61)
    B = workloads.rhs(n, 2, seed=62)
    f = rmge.factor(dev(A), kind=rmge.GAUSSIAN, seed=63, block=128, prec=rmge.F32_BF16X2,
                    pivot=rmge.PIVOT_BLOCK)
    assert f.ok, f.status
    X2, _ = f.solve(dev(B), max_refine=0)                               # FP32 copy
    X1, _ = f.solve(dev(np.ascontiguousarray(B[:, :1])), max_refine=0)  # BF16 copy
    xt = np.linalg.solve(A, B)
    for x, want in ((host(X2)[:, 0], xt[:, 0]), (host(X2)[:, 1], xt[:, 1]),
                    (host(X1)[:, 0], xt[:, 0])):
        err = np.abs(x - want).max() / np.abs(want).max()
        assert err <= 2e-2, err


def test_split16_refactor_reuses_workspaces(rmge):
    # A handle re-factored with a second matrix gives the factors a fresh
    # handle gives (every kernel of the path is deterministic): the BF16
    # operand slabs, the transposed H and the update's term slabs are rewritten
    # where they are read, whatever the first factorization left in them.
    n = 2300
    A1 = workloads.conditioned(n, 1e2, seed=71)
    A2 = workloads.conditioned(n, 1e3, seed=72)
    f = rmge.factor(dev(A1), kind=rmge.GAUSSIAN, seed=73, block=128, prec=rmge.F32_BF16X2,
                    pivot=rmge.PIVOT_BLOCK)
    assert f.ok
    f.refactor(dev(A2))
    assert f.ok
    g = rmge.factor(dev(A2), kind=rmge.GAUSSIAN, seed=73, block=128, prec=rmge.F32_BF16X2,
                    pivot=rmge.PIVOT_BLOCK)
    assert g.ok
    np.testing.assert_array_equal(host(f.lu()), host(g.lu()))
    np.testing.assert_array_equal(host(f.perm()), host(g.perm()))
