"""The synthetic input recipes (host logic, no method arithmetic).

The batch generator builds A_s = Q1 diag(sigma) Q2^T from Haar factors made by
CholeskyQR2 over padded groups of orders; its singular values must be the
stated profile (so each system has the condition number the table gives), and
the padding must not leak into a system.
"""
import numpy as np
import pytest

import workloads


def _reoffset(table):
    out, ao, vo = [], 0, 0
    for t in table:
        out.append((t[0], t[1], t[2], ao, vo, t[5]))
        ao += t[0] * t[0]
        vo += t[0]
    return out


@pytest.mark.parametrize("n_lo,n_hi,count", [(1, 70, 24), (5, 200, 30)])
def test_batch_inputs_have_the_stated_singular_values(n_lo, n_hi, count):
    table = workloads.batch_table(count, 3, n_lo=n_lo, n_hi=n_hi)
    A, B = workloads.batch_inputs_torch(table, 3, device="cpu")
    assert A.numel() == sum(t[0] ** 2 for t in table)
    assert B.numel() == sum(t[0] for t in table)
    for n, kind, seed, ao, vo, kappa in table:
        M = A[ao:ao + n * n].reshape(n, n).numpy()
        s = np.linalg.svd(M, compute_uv=False)
        want = np.sort(workloads.sigma_profile(n, kappa))[::-1]
        assert np.abs(s - want).max() <= 1e-13 * want.max(), (n, kappa)


def test_batch_inputs_large_orders_and_determinism():
    table = _reoffset([t for t in workloads.batch_table(64, 5) if t[0] > 900][:2])
    A1, _ = workloads.batch_inputs_torch(table, 5, device="cpu")
    A2, _ = workloads.batch_inputs_torch(table, 5, device="cpu")
    assert (A1 == A2).all()
    for n, kind, seed, ao, vo, kappa in table:
        M = A1[ao:ao + n * n].reshape(n, n).numpy()
        s = np.linalg.svd(M, compute_uv=False)
        want = np.sort(workloads.sigma_profile(n, kappa))[::-1]
        assert np.abs(s - want).max() <= 1e-13 * want.max()
        assert np.linalg.cond(M) == pytest.approx(kappa, rel=1e-6)
