"""Pins for the oracle's multipliers and the preprocessing product M = A H.

* Circulant: Theorem thcpw gives C = Omega^{-1} diag(Omega c) Omega with the DFT
  matrix Omega = (omega^{ij}), omega = exp(2 pi sqrt(-1) / n) (Section 6).  The
  test builds Omega from that definition and checks the oracle's dense C.
* Circulant and Toeplitz against scipy's independent constructors, and the
  Toeplitz multiplier as the leading n x n block of a (2n-1)-circulant.
* The dense product against exact integer arithmetic.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads


@pytest.mark.parametrize("n", [1, 2, 5, 16, 33])
def test_circulant_closed_form(orc, n):
    c = orc.multiplier_params(orc.CIRCULANT, n, seed=11)
    C = orc.multiplier_dense(orc.CIRCULANT, n, c)
    idx = np.arange(n)
    Omega = np.exp(2j * np.pi * np.outer(idx, idx) / n)
    u = Omega @ c
    closed = np.linalg.inv(Omega) @ np.diag(u) @ Omega
    np.testing.assert_allclose(C, closed.real, atol=1e-12 * max(1, n))
    assert np.max(np.abs(closed.imag)) < 1e-12 * max(1, n)
    # and its inverse by the same theorem
    Cinv = np.linalg.inv(Omega) @ np.diag(1.0 / u) @ Omega
    np.testing.assert_allclose(C @ Cinv.real, np.eye(n), atol=1e-9)


@pytest.mark.parametrize("n", [1, 3, 8, 31])
def test_circulant_matches_scipy(orc, n):
    c = orc.multiplier_params(orc.CIRCULANT, n, seed=3)
    np.testing.assert_array_equal(orc.multiplier_dense(orc.CIRCULANT, n, c), sla.circulant(c))


@pytest.mark.parametrize("n", [1, 2, 7, 32])
def test_toeplitz_layout(orc, n):
    tau = orc.multiplier_params(orc.TOEPLITZ, n, seed=9)
    assert tau.size == 2 * n - 1
    T = orc.multiplier_dense(orc.TOEPLITZ, n, tau)
    first_col = tau[:n]
    first_row = np.concatenate([[tau[0]], tau[n:]])
    np.testing.assert_array_equal(T, sla.toeplitz(first_col, first_row))
    # leading n x n block of the circulant with first column (t_0..t_{n-1}, t_{-(n-1)}..t_{-1})
    col = np.concatenate([tau[:n], tau[n:][::-1]])
    np.testing.assert_array_equal(T, sla.circulant(col)[:n, :n])


def test_gaussian_is_row_major_stream(orc):
    n = 9
    G = orc.multiplier(orc.GAUSSIAN, n, seed=4)
    np.testing.assert_array_equal(G.ravel(), orc.normals(4, 1, n * n))


def test_identity_for_none(orc):
    np.testing.assert_array_equal(orc.multiplier(orc.NONE, 5, 0), np.eye(5))


@pytest.mark.parametrize("shape", [(1, 1, 1), (5, 7, 3), (40, 33, 29)])
def test_matmul_exact_on_integers(orc, shape):
    m, q, p = shape
    rng = np.random.default_rng(1)
    A = rng.integers(-50, 51, size=(m, q))
    B = rng.integers(-50, 51, size=(q, p))
    want = A.astype(np.int64) @ B.astype(np.int64)
    got = orc.matmul(A.astype(float), B.astype(float))
    np.testing.assert_array_equal(got, want.astype(float))


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_preprocessed_product_fft(orc, kind):
    """A H for structured H equals the row-wise FFT correlation (the fast route)."""
    n = 64
    A = workloads.conditioned(n, 1e3, seed=2)
    H = orc.multiplier(kind, n, seed=21)
    M = orc.matmul(A, H)
    if kind == 2:
        c = orc.multiplier_params(kind, n, 21)
        fast = np.fft.ifft(np.fft.fft(A, axis=1) * np.conj(np.fft.fft(c))[None, :], axis=1).real
        np.testing.assert_allclose(M, fast, atol=1e-13 * np.abs(A).max() * np.abs(c).sum())
    else:
        np.testing.assert_allclose(M, A @ H, rtol=0, atol=1e-12 * np.abs(A).max() * np.abs(H).max() * n)
