"""Seeded synthetic inputs shaped like the paper's test matrices.

This module holds only input generation: random orthogonal factors, singular
value profiles, right-hand sides.  It contains none of the method's arithmetic
(no multiplier, no elimination, no solve), and both the GPU tests and the CPU
oracle draw their inputs from it.

Recipes (Pan, Qian, Yan, arXiv:1406.5802, Section 8.1 builds test matrices as
U Sigma V^T with U, V the Q factors of QR factorizations of random matrices):

* ``haar(n, rng)``: Q of a Gaussian matrix with the diagonal of R made
  positive, which makes Q Haar-distributed.
* ``conditioned(n, kappa, seed)``: Q1 diag(sigma) Q2^T with
  sigma_i = kappa^(-i/(n-1)), so ||A||_2 = 1 and kappa_2(A) = kappa exactly
  (up to the rounding of the product).
* ``breakdown_case(seed)``: n = 256, kappa = 1e4, then row 63 of the leading
  64 x 64 block is zeroed (entries A[63, 0:64]); the leading 64 x 64 block is
  singular while A stays nonsingular, so plain GENP meets an exactly zero pivot.
* ``paper_e1(n, seed)``: the Section 8.1 family A = [[A_k, B], [C, D]] with
  k = n/2, A_k = U diag(1,..,1,0,0,0,0) V^T (nullity 4) and B, C, D Gaussian
  Toeplitz matrices scaled to unit spectral norm.
* ``precision_kappa(seed)``: kappa = 10^(1 + 7 u), u uniform on [0, 1).
* ``rhs(n, nrhs, seed)``: i.i.d. N(0, 1).
* ``gaussian_torch(n, seed)``: an i.i.d. N(0, 1/n) matrix made on the GPU with
  no factorization; used where only the shape matters (hardware counters).
* ``batch_table(count, seed)``: the batching workload's systems: orders
  uniform on {32, ..., 1024}, multiplier kind Gaussian or circulant with
  probability 1/2 each, kappa = 10^(1 + 5 u), a multiplier seed each, and the
  offsets of each A_s (n x n, row-major) and b_s, x_s in flat buffers;
  ``batch_inputs_torch(table, seed)`` builds the matrices on the GPU as
  ``conditioned`` does (the Q factors of Gaussian matrices by CholeskyQR2,
  batched over orders within 64 of each other) and the right-hand sides.

The torch variants build the same recipes on a GPU for sizes where a CPU QR
would take minutes; they are not bitwise equal to the numpy ones.
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int, salt: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(salt)])


def haar(n: int, rng: np.random.Generator) -> np.ndarray:
    X = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(X)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :]


def sigma_profile(n: int, kappa: float) -> np.ndarray:
    if n == 1:
        return np.ones(1)
    return float(kappa) ** (-np.arange(n, dtype=np.float64) / (n - 1))


def conditioned(n: int, kappa: float, seed: int) -> np.ndarray:
    rng = _rng(seed, 1)
    Q1 = haar(n, rng)
    Q2 = haar(n, rng)
    return (Q1 * sigma_profile(n, kappa)[None, :]) @ Q2.T


def breakdown_case(seed: int, n: int = 256, kappa: float = 1e4, lead: int = 64) -> np.ndarray:
    A = conditioned(n, kappa, seed)
    A[lead - 1, 0:lead] = 0.0
    return A


def _toeplitz_gaussian(m: int, rng: np.random.Generator) -> np.ndarray:
    t = rng.standard_normal(2 * m - 1)
    idx = np.arange(m)[:, None] - np.arange(m)[None, :]
    T = t[idx + (m - 1)]
    return T / np.linalg.norm(T, 2)


def paper_e1(n: int, seed: int) -> np.ndarray:
    k = n // 2
    rng = _rng(seed, 2)
    U = haar(k, rng)
    V = haar(k, rng)
    s = np.ones(k)
    s[k - 4:] = 0.0
    Ak = (U * s[None, :]) @ V.T
    B = _toeplitz_gaussian(k, rng)
    C = _toeplitz_gaussian(k, rng)
    D = _toeplitz_gaussian(k, rng)
    return np.block([[Ak, B], [C, D]])


def precision_kappa(seed: int) -> float:
    return float(10.0 ** (1.0 + 7.0 * _rng(seed, 3).random()))


def rhs(n: int, nrhs: int, seed: int) -> np.ndarray:
    return _rng(seed, 4).standard_normal((n, nrhs))


def integer_matrix(n: int, seed: int, lo: int = -3, hi: int = 3) -> np.ndarray:
    """Small-integer matrix (exact-arithmetic tests)."""
    return _rng(seed, 5).integers(lo, hi + 1, size=(n, n)).astype(np.float64)


# ---------------------------------------------------------------------------
# GPU-side generation of the same recipes for large n (torch, seeded).
# ---------------------------------------------------------------------------

def conditioned_torch(n: int, kappa: float, seed: int, device="cuda"):
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed) * 1000003 + 17)

    def _haar():
        X = torch.randn((n, n), generator=g, dtype=torch.float64, device=device)
        Q, R = torch.linalg.qr(X)
        s = torch.sign(torch.diagonal(R))
        s[s == 0] = 1.0
        return Q * s[None, :]

    Q1 = _haar()
    Q2 = _haar()
    sig = torch.as_tensor(sigma_profile(n, kappa), dtype=torch.float64, device=device)
    A = torch.matmul(Q1 * sig[None, :], Q2.T.contiguous())
    del Q1, Q2
    return A.contiguous()


def gaussian_torch(n: int, seed: int, device="cuda"):
    """i.i.d. N(0, 1) n x n matrix, scaled by 1/sqrt(n) (kappa grows like n)."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed) * 1000003 + 41)
    A = torch.randn((n, n), generator=g, dtype=torch.float64, device=device)
    return A.mul_(1.0 / float(n) ** 0.5)


def rhs_torch(n: int, nrhs: int, seed: int, device="cuda"):
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed) * 1000003 + 29)
    return torch.randn((n, nrhs), generator=g, dtype=torch.float64, device=device)


def batch_table(count: int, seed: int, n_lo: int = 32, n_hi: int = 1024,
                log_kappa: tuple = (1.0, 6.0)) -> list:
    """(n, kind, multiplier seed, a_off, v_off, kappa) for each system (kind 1
    Gaussian, 2 circulant)."""
    rng = _rng(seed, 7)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    kinds = np.where(rng.random(count) < 0.5, 1, 2)
    kappas = 10.0 ** (log_kappa[0] + (log_kappa[1] - log_kappa[0]) * rng.random(count))
    out, a_off, v_off = [], 0, 0
    for i in range(count):
        n = int(ns[i])
        out.append((n, int(kinds[i]), int(seed) * 100003 + i, a_off, v_off, float(kappas[i])))
        a_off += n * n
        v_off += n
    return out


def batch_inputs_torch(table, seed: int, device="cuda"):
    """Flat float64 tensors A (every A_s row-major at its offset) and B (every
    b_s), built on the GPU: A_s = Q1 diag(sigma) Q2^T with Haar Q1, Q2.  The Q
    factor of a Gaussian X with R's diagonal positive is X R^{-1} with R the
    Cholesky factor of X^T X; done twice (CholeskyQR2) it is orthogonal to
    working precision, and batched over groups of orders within 64 of each
    other: X_s padded to the group's order P as [[X_s, 0], [0, I]] has the
    factor [[Q_s, 0], [0, I]]."""
    import torch

    a_total = sum(t[0] * t[0] for t in table)
    v_total = sum(t[0] for t in table)
    A = torch.empty(a_total, dtype=torch.float64, device=device)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) * 1000003 + 53)
    groups = {}
    for i, t in enumerate(table):
        groups.setdefault((t[0] + 63) // 64, []).append(i)

    def _inv_upper(R):
        # R^{-1} for a batch of upper-triangular R (order a multiple of 32) with
        # batched products only: the 32 x 32 diagonal blocks are inverted by
        # substitution all at once, then the block rows of R^{-1} follow from
        # the bottom up, X_I = R_II^{-1} (E_I - R_{I,>I} X_{>I}).  (The library
        # triangular solve needs a larger workspace than the BLAS handle has
        # for batches of large orders.)
        k, P, _ = R.shape
        q = P // 32
        D = R.reshape(k, q, 32, q, 32).diagonal(dim1=1, dim2=3).permute(0, 3, 1, 2)
        D = D.reshape(k * q, 32, 32)
        Y = torch.zeros_like(D)
        eye = torch.eye(32, dtype=R.dtype, device=R.device)
        for i in range(31, -1, -1):
            row = eye[i].expand(k * q, 32)
            if i < 31:
                row = row - (D[:, i:i + 1, i + 1:] @ Y[:, i + 1:, :])[:, 0, :]
            Y[:, i, :] = row / D[:, i, i:i + 1]
        Y = Y.reshape(k, q, 32, 32)
        X = torch.zeros_like(R)
        for I in range(q - 1, -1, -1):
            r0, r1 = 32 * I, 32 * I + 32
            rhs = torch.zeros((k, 32, P - r0), dtype=R.dtype, device=R.device)
            rhs[:, :, :32] = eye
            if r1 < P:
                rhs[:, :, 32:] -= R[:, r0:r1, r1:] @ X[:, r1:, r1:]
            X[:, r0:r1, r0:] = Y[:, I] @ rhs
        return X

    def _chol_qr(X):
        R = torch.linalg.cholesky(X.transpose(1, 2).contiguous() @ X, upper=True)
        return X @ _inv_upper(R)

    for key in sorted(groups):
        P = 64 * key
        for c0 in range(0, len(groups[key]), 128):  # bounded memory: 128 x P^2 doubles a chunk
            idx = groups[key][c0:c0 + 128]
            k = len(idx)
            ns = torch.tensor([table[i][0] for i in idx], device=device)
            ar = torch.arange(P, device=device)
            keep = (ar[None, :, None] < ns[:, None, None]) & (ar[None, None, :] < ns[:, None, None])
            pad_eye = ((ar[None, :, None] >= ns[:, None, None]) &
                       (ar[None, :, None] == ar[None, None, :])).to(torch.float64)

            def _haar():
                X = torch.randn((k, P, P), generator=g, dtype=torch.float64, device=device)
                X = X * keep + pad_eye
                return _chol_qr(_chol_qr(X))

            Q1, Q2 = _haar(), _haar()
            for j, i in enumerate(idx):
                n = table[i][0]
                sig = torch.as_tensor(sigma_profile(n, table[i][5]), device=device)
                As = (Q1[j, :n, :n] * sig[None, :]) @ Q2[j, :n, :n].transpose(0, 1).contiguous()
                off = table[i][3]
                A[off:off + n * n] = As.reshape(-1)
            del Q1, Q2
    gb = torch.Generator(device=device)
    gb.manual_seed(int(seed) * 1000003 + 59)
    B = torch.randn(v_total, generator=gb, dtype=torch.float64, device=device)
    return A, B
