"""The Schur-complement update on the BF16 matrix cores, and BF16 factors.

1. One update C <- C - D E (eq. eqgenp), through rmge_schur_update_f32, against
   the FP64 product on the host, elementwise:
   * FP32 matrix cores and the three-term BF16 split (precision F32_BF16X2)
     both meet the FP32 bound |C_g - (C - D E)| <= (K + 3) 2^-24 (|C| + |D| |E|):
     K + 1 FP32 roundings of the accumulation, and for the split the three
     dropped cross products, at most (2^-24 + 2^-34) |d e| each;
   * the one-term update of the BF16 factors (operands rounded once to BF16,
     2^-9 relative each) meets (2^-8 + 2^-18) |D| |E| on top of that, and does
     NOT meet the FP32 bound -- which shows the FP32 check above would catch a
     split that lost its second and third terms.
2. BF16 factors (precision BF16): L U reproduces M = A H up to the BF16
   operand rounding of each bulk update, ||L U - M||_max <= (2^-8 + 2^-18) *
   (number of updates) * || |L| |U| ||_max plus the FP32 factor bound; with a
   FP64 GMRES refinement the reported backward error is the true one of the
   returned x, converged or not (the BF16 factors' error, 2^-9 times the
   growth, is too large for refinement to recover at larger n).
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


def _update(rmge, M, N, K, terms, seed, scale_e=1.0):
    import torch

    rng = np.random.default_rng(seed)
    D = rng.standard_normal((M, K)).astype(np.float32)
    E = (scale_e * rng.standard_normal((K, N))).astype(np.float32)
    C = rng.standard_normal((M, N)).astype(np.float32)
    Cd = torch.as_tensor(C, device="cuda").clone()
    rmge.schur_update(Cd, torch.as_tensor(D, device="cuda"), torch.as_tensor(E, device="cuda"),
                      terms)
    got = Cd.cpu().numpy().astype(np.float64)
    D64, E64, C64 = (x.astype(np.float64) for x in (D, E, C))
    want = C64 - D64 @ E64
    mag = np.abs(D64) @ np.abs(E64)
    return got, want, np.abs(C64), mag


# ragged tiles (M, N not multiples of 256), depths that are not whole 32-wide
# chunks, and a 2304-wide block of full tiles
SHAPES = [(1000, 777, 256), (2304, 2304, 256), (513, 300, 100), (256, 4000, 32), (70, 90, 7)]


@pytest.mark.parametrize("M,N,K", SHAPES)
@pytest.mark.parametrize("terms", [0, 3])
def test_update_fp32_accuracy(rmge, M, N, K, terms):
    got, want, cabs, mag = _update(rmge, M, N, K, terms, seed=M + N + K)
    bound = (K + 3) * U32 * (cabs + mag)
    ratio = float((np.abs(got - want) / bound).max())
    assert ratio <= 1.0, ratio


@pytest.mark.parametrize("M,N,K", SHAPES[:3])
def test_update_one_term_bf16_accuracy_and_teeth(rmge, M, N, K):
    got, want, cabs, mag = _update(rmge, M, N, K, 1, seed=7 * M + K)
    err = np.abs(got - want)
    fp32_bound = (K + 3) * U32 * (cabs + mag)
    bf16_bound = (2.0 ** -8 + 2.0 ** -18) * mag + fp32_bound
    assert (err <= bf16_bound).all(), float((err / bf16_bound).max())
    # a one-term product is far outside the FP32 bound that the split meets
    assert float((err / fp32_bound).max()) > 4.0


@pytest.mark.parametrize("terms", [0, 1, 3])
def test_update_wide_dynamic_range(rmge, terms):
    # E spanning 2^-20 .. 2^20: the split's terms are relative to each value,
    # so the FP32 bound holds whatever the magnitudes
    got, want, cabs, mag = _update(rmge, 600, 520, 256, terms, seed=3, scale_e=2.0 ** 20)
    K = 256
    bound = (K + 3) * U32 * (cabs + mag)
    if terms == 1:
        bound = bound + (2.0 ** -8 + 2.0 ** -18) * mag
    assert (np.abs(got - want) <= bound).all()


def test_update_rejects_bad_arguments(rmge):
    import torch

    from paper_1406_5802_amd import _rmge

    x = torch.zeros((4, 4), dtype=torch.float32, device="cuda")
    p = x.data_ptr()
    s = int(torch.cuda.current_stream().cuda_stream)
    assert _rmge.rmge_schur_update_f32(4, 4, 4, p, 4, p, 4, p, 4, 2, s) == _rmge.RMGE_EINVAL
    assert _rmge.rmge_schur_update_f32(4, 4, 300, p, 300, p, 4, p, 4, 3, s) == _rmge.RMGE_EINVAL
    assert _rmge.rmge_schur_update_f32(4, 4, 4, p, 3, p, 4, p, 4, 3, s) == _rmge.RMGE_EINVAL


@pytest.mark.parametrize("kind", ["UNITARY_CIRCULANT", "GAUSSIAN"])
@pytest.mark.parametrize("n,block", [(600, 256), (1300, 128), (2200, 256)])
def test_bf16_factors_backward_error(rmge, kind, n, block):
    A = workloads.conditioned(n, 1e1, seed=81)
    k = getattr(rmge, kind)
    f = rmge.factor(dev(A), kind=k, seed=83, block=block, prec=rmge.BF16)
    assert f.ok, f.status
    H = oracle.multiplier(k, n, 83)
    if kind == "GAUSSIAN":  # the product runs with H rounded to BF16 (as F32_BF16X2)
        from test_gpu_split16 import _bf16

        H = _bf16(H)
    Mo = oracle.matmul(A, H)
    LU = host(f.lu())
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    back = np.abs(L @ U - Mo).max()
    lu_abs = (np.abs(L) @ np.abs(U)).max()
    updates = max(1, -(-n // block) - 1)
    mdiff = (2.0 ** -17 + 2 * (n + 4) * U32) * (np.abs(A) @ np.abs(H)).max()
    bound = ((2.0 ** -8 + 2.0 ** -18) * updates + 8 * n * U32 * _kappa32(L, U)) * lu_abs + mdiff
    assert back <= bound, (back, bound)
    # and they are BF16-level, not FP32-level, factors (the updates did round)
    if n >= 1300:
        assert back > 8 * n * U32 * (np.abs(L) @ np.abs(U)).max() / 64


@pytest.mark.parametrize("n", [96, 512])
def test_bf16_factors_gmres_reports_its_error(rmge, n):
    # BF16 factors carry 2^-9 times the growth as backward error, so FP64 GMRES
    # refinement preconditioned by them reaches 1e-14 only for small n (the
    # result is stated per solve, converged or not): the reported eta must be
    # the normwise backward error of the returned x, recomputed here, and the
    # converged flag must agree with it.  Where it converges, x matches the
    # oracle's solution.
    A = workloads.conditioned(n, 1e1, seed=91)
    B = workloads.rhs(n, 1, seed=92)
    f = rmge.factor(dev(A), kind=rmge.UNITARY_CIRCULANT, seed=93, block=32, prec=rmge.BF16)
    assert f.ok
    X, st = f.solve_gmres(dev(B), max_iters=300, restart=32, tol=1e-14)
    x = host(X)[:, 0]
    r = B[:, 0] - A @ x
    eta = np.abs(r).max() / (np.abs(A).sum(axis=1).max() * np.abs(x).max() + np.abs(B).max())
    assert np.isfinite(st["eta"])
    assert eta == pytest.approx(st["eta"], rel=0.1, abs=1e-16)
    assert bool(st["converged"]) == (st["eta"] <= 1e-14)
    if st["converged"]:
        so = oracle.solve(oracle.factor(A, oracle.UNITARY_CIRCULANT, 93), B, refine=1)
        rel = np.linalg.norm(host(X) - so.X) / np.linalg.norm(so.X)
        assert rel <= max(1e-10, 2 * 10 * (st["eta"] + so.eta[-1])), rel
