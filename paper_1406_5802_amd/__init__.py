"""Random-multiplier Gaussian elimination with no pivoting on MI355X (gfx950).

Python side of ``librmge.so`` (include/rmge.h).  It only marshals arguments:
PyTorch supplies device memory and the stream, and every step of the method
(multiplier generation, M = A H, block elimination, solves, refinement,
adjoint) runs in the library's HIP kernels.

    import torch, paper_1406_5802_amd as rmge
    f = rmge.factor(A, kind=rmge.GAUSSIAN, seed=1, block=256)   # A: cuda float64, n x n
    X, st = f.solve(B, max_refine=1)                              # X = A^{-1} B
    Y = f.solve_adjoint(W)                                        # Y = A^{-T} W
"""
from __future__ import annotations

from . import _rmge
from ._rmge import (RMGE_F32, RMGE_F32_BF16X2, RMGE_F64, RMGE_MULT_CIRCULANT, RMGE_MULT_GAUSSIAN,
                    RMGE_MULT_NONE, RMGE_MULT_TOEPLITZ, RMGE_PIVOT_BLOCK, RMGE_PIVOT_NONE,
                    RMGEError, lib)

NONE, GAUSSIAN, CIRCULANT, TOEPLITZ = (RMGE_MULT_NONE, RMGE_MULT_GAUSSIAN, RMGE_MULT_CIRCULANT,
                                       RMGE_MULT_TOEPLITZ)
F64, F32 = RMGE_F64, RMGE_F32
# FP32 factors with the product A H on the BF16 matrix cores (H rounded to BF16,
# A split into two BF16 terms); other multiplier kinds behave as F32
F32_BF16X2 = RMGE_F32_BF16X2
PIVOT_NONE, PIVOT_BLOCK = RMGE_PIVOT_NONE, RMGE_PIVOT_BLOCK
KIND_NAMES = {"none": NONE, "gaussian": GAUSSIAN, "circulant": CIRCULANT, "toeplitz": TOEPLITZ}


def _stream_handle(device) -> int:
    import torch

    return int(torch.cuda.current_stream(device).cuda_stream)


def _check_matrix(A, name="A"):
    import torch

    if not isinstance(A, torch.Tensor) or A.device.type != "cuda":
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if A.dtype != torch.float64:
        raise TypeError("%s must be float64" % name)
    if A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("%s must be a row-major 2-D tensor" % name)


def _kind(kind) -> int:
    if isinstance(kind, str):
        return KIND_NAMES[kind.lower()]
    return int(kind)


class Factors:
    """A factorization handle: owns L, U and the multiplier; borrows A."""

    def __init__(self, A, kind=GAUSSIAN, seed=0, block=256, prec=F64, pivot=PIVOT_NONE):
        _check_matrix(A)
        n = A.shape[0]
        if A.shape[1] != n:
            raise ValueError("A must be square")
        self.A = A  # kept alive: the library reads it during refinement
        self.n, self.kind, self.seed, self.block, self.prec = n, _kind(kind), seed, block, prec
        self.pivot = pivot
        self.device = A.device
        rc, h = _rmge.rmge_factor_pivoted(A.data_ptr(), n, A.stride(0), self.kind, seed, block,
                                          prec, pivot, _stream_handle(A.device))
        if rc not in (_rmge.RMGE_OK, _rmge.RMGE_ZERO_PIVOT, _rmge.RMGE_NONFINITE):
            raise RMGEError(rc, "rmge_factor_ex")
        self._h = h
        self.status = rc

    @property
    def ok(self) -> bool:
        return self.status == _rmge.RMGE_OK

    def refactor(self, A, seed=None):
        _check_matrix(A)
        if tuple(A.shape) != (self.n, self.n):
            raise ValueError("shape mismatch")
        self.A = A
        if seed is not None:
            self.seed = seed
        rc = _rmge.rmge_refactor(self._h, A.data_ptr(), A.stride(0), self.seed)
        if rc not in (_rmge.RMGE_OK, _rmge.RMGE_ZERO_PIVOT, _rmge.RMGE_NONFINITE):
            raise RMGEError(rc, "rmge_refactor")
        self.status = rc
        return rc

    def stats(self):
        rc, st = _rmge.rmge_factor_stats_get(self._h)
        if rc:
            raise RMGEError(rc, "rmge_factor_stats_get")
        return {"info": st.info, "status": st.status, "block": st.block,
                "min_abs_pivot": st.min_abs_pivot, "growth": st.growth,
                "ms_multiplier": st.ms_multiplier, "ms_product": st.ms_product,
                "ms_factor": st.ms_factor}

    def times(self):
        """Phase times (ms) of the last factorization, with no device work."""
        rc, ms = _rmge.rmge_factor_times(self._h)
        if rc:
            raise RMGEError(rc, "rmge_factor_times")
        return {"ms_multiplier": ms[0], "ms_product": ms[1], "ms_factor": ms[2]}

    @property
    def info(self) -> int:
        return self.stats()["info"]

    def solve(self, B, max_refine=1, tol=0.0, out=None, raise_on_not_converged=False):
        """X = A^{-1} B (B: n or n x nrhs, float64 CUDA).  Returns (X, stats dict)."""
        import torch

        vec = B.dim() == 1
        B2 = B.reshape(-1, 1) if vec else B
        _check_matrix(B2, "B")
        nrhs = B2.shape[1]
        X = out if out is not None else torch.empty((self.n, nrhs), dtype=torch.float64,
                                                    device=B.device)
        rc, st = _rmge.rmge_solve(self._h, B2.data_ptr(), nrhs, B2.stride(0), X.data_ptr(),
                                  X.stride(0), max_refine, tol)
        if rc not in (_rmge.RMGE_OK, _rmge.RMGE_NOT_CONVERGED) or (
                raise_on_not_converged and rc == _rmge.RMGE_NOT_CONVERGED):
            raise RMGEError(rc, "rmge_solve")
        stats = {"status": rc, "iters": st.iters, "converged": bool(st.converged),
                 "eta0": st.eta0, "eta": st.eta,
                 "eta_hist": [st.eta_hist[i] for i in range(st.iters + 1)]}
        return (X.reshape(-1) if vec else X), stats

    def solve_gmres(self, B, max_iters=200, restart=32, tol=1e-14, out=None,
                    raise_on_not_converged=False, trans=False):
        """X = A^{-1} B (A^{-T} B with trans) with GMRES-based refinement preconditioned by
        the factors."""
        import torch

        vec = B.dim() == 1
        B2 = B.reshape(-1, 1) if vec else B
        _check_matrix(B2, "B")
        nrhs = B2.shape[1]
        X = out if out is not None else torch.empty((self.n, nrhs), dtype=torch.float64,
                                                    device=B.device)
        rc, st = _rmge.rmge_solve_gmres(self._h, 1 if trans else 0, B2.data_ptr(), nrhs,
                                        B2.stride(0), X.data_ptr(), X.stride(0), max_iters,
                                        restart, tol)
        if rc not in (_rmge.RMGE_OK, _rmge.RMGE_NOT_CONVERGED) or (
                raise_on_not_converged and rc == _rmge.RMGE_NOT_CONVERGED):
            raise RMGEError(rc, "rmge_solve_gmres")
        nh = min(17, max(1, sum(1 for i in range(17) if st.eta_hist[i] != 0.0)))
        stats = {"status": rc, "iters": st.iters, "converged": bool(st.converged),
                 "eta0": st.eta0, "eta": st.eta, "eta_hist": [st.eta_hist[i] for i in range(nh)]}
        return (X.reshape(-1) if vec else X), stats

    def solve_adjoint(self, W, out=None):
        """Y = A^{-T} W."""
        import torch

        vec = W.dim() == 1
        W2 = W.reshape(-1, 1) if vec else W
        _check_matrix(W2, "W")
        nrhs = W2.shape[1]
        Y = out if out is not None else torch.empty((self.n, nrhs), dtype=torch.float64,
                                                    device=W.device)
        rc = _rmge.rmge_solve_adjoint(self._h, W2.data_ptr(), nrhs, W2.stride(0), Y.data_ptr(),
                                      Y.stride(0))
        if rc:
            raise RMGEError(rc, "rmge_solve_adjoint")
        return Y.reshape(-1) if vec else Y

    def solve_adjoint_refined(self, W, max_refine=16, tol=1e-14, out=None):
        """Y = A^{-T} W with FP64 refinement.  Returns (Y, stats dict)."""
        import torch

        vec = W.dim() == 1
        W2 = W.reshape(-1, 1) if vec else W
        _check_matrix(W2, "W")
        nrhs = W2.shape[1]
        Y = out if out is not None else torch.empty((self.n, nrhs), dtype=torch.float64,
                                                    device=W.device)
        rc, st = _rmge.rmge_solve_adjoint_ex(self._h, W2.data_ptr(), nrhs, W2.stride(0),
                                             Y.data_ptr(), Y.stride(0), max_refine, tol)
        if rc not in (_rmge.RMGE_OK, _rmge.RMGE_NOT_CONVERGED):
            raise RMGEError(rc, "rmge_solve_adjoint_ex")
        stats = {"status": rc, "iters": st.iters, "converged": bool(st.converged),
                 "eta0": st.eta0, "eta": st.eta,
                 "eta_hist": [st.eta_hist[i] for i in range(st.iters + 1)]}
        return (Y.reshape(-1) if vec else Y), stats

    def lu(self):
        """Packed factors as an n x n float64 tensor (unit L below, U on and above)."""
        import torch

        LU = torch.empty((self.n, self.n), dtype=torch.float64, device=self.device)
        rc = _rmge.rmge_factors_lu(self._h, LU.data_ptr(), LU.stride(0))
        if rc:
            raise RMGEError(rc, "rmge_factors_lu")
        return LU

    def perm(self):
        """Row order of the factors (int32 tensor): row t of L U is row perm[t] of A H."""
        import torch

        p = torch.empty(self.n, dtype=torch.int32, device=self.device)
        rc = _rmge.rmge_factors_perm(self._h, p.data_ptr())
        if rc:
            raise RMGEError(rc, "rmge_factors_perm")
        return p

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _rmge.rmge_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def factor(A, kind=GAUSSIAN, seed=0, block=256, prec=F64, pivot=PIVOT_NONE) -> Factors:
    return Factors(A, kind=kind, seed=seed, block=block, prec=prec, pivot=pivot)


def multiplier_params(kind, n, seed, device="cuda"):
    """The multiplier's random parameters as the library draws them (float64 CUDA tensor)."""
    import torch

    kind = _kind(kind)
    cnt = _rmge.rmge_param_count(kind, n)
    out = torch.empty(cnt, dtype=torch.float64, device=device)
    rc = _rmge.rmge_multiplier_params(kind, n, seed, out.data_ptr(),
                                      _stream_handle(out.device))
    if rc:
        raise RMGEError(rc, "rmge_multiplier_params")
    return out


def precondition(A, kind, seed):
    """M = A H in FP64 (the preprocessing product alone)."""
    import torch

    _check_matrix(A)
    n = A.shape[0]
    M = torch.empty((n, n), dtype=torch.float64, device=A.device)
    rc = _rmge.rmge_precondition(A.data_ptr(), n, A.stride(0), _kind(kind), seed, M.data_ptr(),
                                 M.stride(0), _stream_handle(A.device))
    if rc:
        raise RMGEError(rc, "rmge_precondition")
    return M


def grad_A(GB, X):
    """-GB X^T (the gradient of a loss with respect to A, given GB = A^{-T} dL/dX)."""
    import torch

    n, nrhs = X.shape
    GA = torch.empty((n, n), dtype=torch.float64, device=X.device)
    rc = _rmge.rmge_grad_A(GB.data_ptr(), GB.stride(0), X.data_ptr(), X.stride(0), n, nrhs,
                           GA.data_ptr(), GA.stride(0), _stream_handle(X.device))
    if rc:
        raise RMGEError(rc, "rmge_grad_A")
    return GA


__all__ = ["factor", "Factors", "multiplier_params", "precondition", "grad_A", "RMGEError", "lib",
           "NONE", "GAUSSIAN", "CIRCULANT", "TOEPLITZ", "F64", "F32", "F32_BF16X2", "PIVOT_NONE",
           "PIVOT_BLOCK"]
