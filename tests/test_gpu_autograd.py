"""Differentiation through the solve: the hand-written adjoint of
paper_1406_5802_amd.autograd (grad_B = A^{-T} grad_X, grad_A = -grad_B X^T) against
the oracle's gradient and against central finite differences (h = 1e-6, FP64), at
small n and at the n = 8192 Toeplitz workload with 16 right-hand sides.

Finite-difference tolerance: the loss L = sum(W .* X) is evaluated with solutions
refined to eta <= 1e-14, so each evaluation carries an error of about
kappa(A) eta |W| |X|; divided by 2h that bounds the difference quotient's noise.
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


def _grads(rmge, A, B, W, **kw):
    import torch

    from paper_1406_5802_amd import autograd

    At = A.clone().requires_grad_(True)
    Bt = B.clone().requires_grad_(True)
    X = autograd.solve(At, Bt, **kw)
    loss = (W * X).sum()
    loss.backward()
    return X.detach(), At.grad, Bt.grad, float(loss.detach())


@pytest.mark.parametrize("kind", ["GAUSSIAN", "CIRCULANT", "TOEPLITZ"])
def test_gradients_match_oracle(rmge, kind):
    n, nrhs = 200, 3
    A = workloads.conditioned(n, 1e2, seed=91)
    B = workloads.rhs(n, nrhs, seed=92)
    W = workloads.rhs(n, nrhs, seed=93)
    k = getattr(rmge, kind)
    X, gA, gB, _ = _grads(rmge, dev(A), dev(B), dev(W), kind=k, seed=3, block=64)
    fo = oracle.factor(A, k, 3)
    Xo = oracle.solve(fo, B, refine=2).X
    gBo = oracle.solve_adjoint(fo, W)
    gAo = oracle.grad_A(gBo, Xo)
    for got, want in ((host(X), Xo), (host(gB), gBo), (host(gA), gAo)):
        rel = np.linalg.norm(got - want) / np.linalg.norm(want)
        assert rel <= 1e-10, rel


def test_grad_a_kernel_matches_outer_product(rmge):
    rng = np.random.default_rng(5)
    # nrhs in each of the kernel's register widths (16, 32, 64), ragged tiles
    for n, nrhs in ((1, 1), (17, 3), (300, 16), (129, 17), (1000, 32), (513, 64), (33, 40)):
        GB = rng.standard_normal((n, nrhs))
        X = rng.standard_normal((n, nrhs))
        GA = host(rmge.grad_A(dev(GB), dev(X)))
        want = -(GB @ X.T)
        np.testing.assert_allclose(GA, want, rtol=0, atol=1e-13 * max(1.0, np.abs(want).max()))


def _fd_check(rmge, A, B, W, gA, gB, kw, kappa, count, seed):
    import torch

    from paper_1406_5802_amd import autograd

    n = A.shape[0]
    h = 1e-6
    rng = np.random.default_rng(seed)
    gAh, gBh = host(gA), host(gB)
    scale = np.sqrt(np.mean(gAh ** 2))

    def loss(Am, Bm):
        with torch.no_grad():
            return float((W * autograd.solve(Am, Bm, **kw)).sum())

    for _ in range(count):
        i, j = (int(v) for v in rng.integers(0, n, 2))
        Ap, Am = A.clone(), A.clone()
        Ap[i, j] += h
        Am[i, j] -= h
        fd = (loss(Ap, B) - loss(Am, B)) / (2 * h)
        assert abs(fd - gAh[i, j]) <= 1e-5 * abs(gAh[i, j]) + 1e-4 * scale, (i, j, fd, gAh[i, j])
    bscale = np.sqrt(np.mean(gBh ** 2))
    for _ in range(count // 4):
        i, r = int(rng.integers(0, n)), int(rng.integers(0, B.shape[1]))
        Bp, Bm = B.clone(), B.clone()
        Bp[i, r] += h
        Bm[i, r] -= h
        fd = (loss(A, Bp) - loss(A, Bm)) / (2 * h)
        assert abs(fd - gBh[i, r]) <= 1e-5 * abs(gBh[i, r]) + 1e-4 * bscale, (i, r, fd)


def test_finite_differences_small(rmge):
    n, nrhs = 160, 2
    A = dev(workloads.conditioned(n, 30.0, seed=94))
    B = dev(workloads.rhs(n, nrhs, seed=95))
    W = dev(workloads.rhs(n, nrhs, seed=96))
    kw = dict(kind=rmge.GAUSSIAN, seed=7, block=32)
    _, gA, gB, _ = _grads(rmge, A, B, W, **kw)
    _fd_check(rmge, A, B, W, gA, gB, kw, 30.0, 32, 1)


@pytest.mark.parametrize("prec", ["F64", "F32"])
def test_finite_differences_toeplitz_n8192(rmge, prec):
    # the differentiation workload: n = 8192, Toeplitz multiplier, 16 right-hand sides,
    # loss sum(w .* x), central differences (h = 1e-6) on 32 random entries of A
    n, nrhs, kappa = 8192, 16, 1e2
    A = workloads.conditioned_torch(n, kappa, seed=8)
    B = workloads.rhs_torch(n, nrhs, seed=8)
    W = workloads.rhs_torch(n, nrhs, seed=9)
    kw = dict(kind=rmge.TOEPLITZ, seed=21, block=256, prec=getattr(rmge, prec),
              pivot=rmge.PIVOT_BLOCK if prec == "F32" else rmge.PIVOT_NONE)
    X, gA, gB, _ = _grads(rmge, A, B, W, **kw)
    # grad_B = A^{-T} W, checked directly against LAPACK
    gBl = np.linalg.solve(host(A).T, host(W))
    rel = np.linalg.norm(host(gB) - gBl) / np.linalg.norm(gBl)
    assert rel <= 1e-10, rel
    _fd_check(rmge, A, B, W, gA, gB, kw, kappa, 32, 2)
