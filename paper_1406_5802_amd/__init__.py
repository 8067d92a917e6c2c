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

import ctypes

from . import _rmge
from ._rmge import (RMGE_BF16, RMGE_F32, RMGE_F32_BF16X2, RMGE_F64, RMGE_MULT_CIRCULANT, RMGE_MULT_GAUSSIAN,
                    RMGE_MULT_NONE, RMGE_MULT_TOEPLITZ, RMGE_MULT_UNITARY_CIRCULANT,
                    RMGE_PIVOT_BLOCK, RMGE_PIVOT_NONE, RMGEError, lib)

NONE, GAUSSIAN, CIRCULANT, TOEPLITZ = (RMGE_MULT_NONE, RMGE_MULT_GAUSSIAN, RMGE_MULT_CIRCULANT,
                                       RMGE_MULT_TOEPLITZ)
UNITARY_CIRCULANT = RMGE_MULT_UNITARY_CIRCULANT
F64, F32 = RMGE_F64, RMGE_F32
# FP32 factors whose large Schur updates run on the BF16 matrix cores in
# three-term split form (FP32 accuracy); with a Gaussian multiplier the product
# A H does too (H rounded to BF16, A split into two BF16 terms)
F32_BF16X2 = RMGE_F32_BF16X2
# BF16 factorization: bulk Schur updates with operands rounded once to BF16,
# FP32 accumulation (the product as for F32_BF16X2)
BF16 = RMGE_BF16
PIVOT_NONE, PIVOT_BLOCK = RMGE_PIVOT_NONE, RMGE_PIVOT_BLOCK
KIND_NAMES = {"none": NONE, "gaussian": GAUSSIAN, "circulant": CIRCULANT, "toeplitz": TOEPLITZ,
              "unitary_circulant": UNITARY_CIRCULANT}


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

    def update_time(self):
        """(ms, flops) of the last factorization's bulk Schur updates on the main
        stream (HIP events around each launch; the columns handed to the
        reserved compute units are not counted), with no device work."""
        rc, ms, fl = _rmge.rmge_factor_update_time(self._h)
        if rc:
            raise RMGEError(rc, "rmge_factor_update_time")
        return ms, fl

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


def schur_update(C, D, E, terms):
    """C <- C - D E in FP32 in place (one Schur-complement update as the
    factorization runs it: terms 0 FP32 matrix cores, 3 three-term BF16 split,
    1 operands rounded to BF16)."""
    M, N = C.shape
    K = D.shape[1]
    rc = _rmge.rmge_schur_update_f32(M, N, K, D.data_ptr(), D.stride(0), E.data_ptr(), E.stride(0),
                                     C.data_ptr(), C.stride(0), terms, _stream_handle(C.device))
    if rc:
        raise RMGEError(rc, "rmge_schur_update_f32")
    return C


class Batch:
    """Many independent systems solved in one device-resident pass (rmge_batch_*).

    systems: list of (n, kind, seed, a_off, v_off); A, B, X are flat float64 CUDA
    tensors holding every A_s (row-major, ld n) and b_s, x_s at those offsets."""

    def __init__(self, systems, tuning=None, restart=16, max_iters=200):
        entries = [_rmge.rmge_batch_system(int(n), _kind(k), int(seed) & (2**64 - 1), int(ao), int(vo))
                   for (n, k, seed, ao, vo) in systems]
        t = None
        if tuning is not None:
            t = _rmge.rmge_batch_tuning((ctypes.c_int32 * _rmge.RMGE_BATCH_BUCKETS)(*tuning))
        rc, h = _rmge.rmge_batch_create(entries, t, restart, max_iters)
        if rc:
            raise RMGEError(rc, "rmge_batch_create")
        self._h = h
        self.count = len(entries)

    def run(self, A, B, X, tol=1e-14, graph=False):
        fn = _rmge.rmge_batch_graph_run if graph else _rmge.rmge_batch_run
        rc = fn(self._h, A.data_ptr(), B.data_ptr(), X.data_ptr(), tol, _stream_handle(A.device))
        if rc:
            raise RMGEError(rc, "rmge_batch_run")
        return X

    def run_timed(self, A, B, X, tol=1e-14):
        """An eager run with HIP events between the phases: (products, factorizations,
        refinement, FP64 fallback) in ms."""
        rc, ms = _rmge.rmge_batch_run_timed(self._h, A.data_ptr(), B.data_ptr(), X.data_ptr(), tol,
                                            _stream_handle(A.device))
        if rc:
            raise RMGEError(rc, "rmge_batch_run_timed")
        return ms

    def results(self, device="cuda"):
        import numpy as np

        c = self.count
        st, it, fb = np.zeros(c, np.int32), np.zeros(c, np.int32), np.zeros(c, np.int32)
        eta, eta0, info = np.zeros(c), np.zeros(c), np.zeros(c, np.int64)
        import torch

        rc = _rmge.rmge_batch_results(self._h, st, eta, eta0, it, info, fb,
                                      _stream_handle(torch.device(device)))
        if rc:
            raise RMGEError(rc, "rmge_batch_results")
        return {"status": st, "eta": eta, "eta0": eta0, "iters": it, "info": info, "fp64": fb}

    def tuning(self):
        rc, nb = _rmge.rmge_batch_get_tuning(self._h)
        if rc:
            raise RMGEError(rc, "rmge_batch_get_tuning")
        return nb

    def set_tuning(self, nb):
        rc = _rmge.rmge_batch_set_tuning(self._h, nb)
        if rc:
            raise RMGEError(rc, "rmge_batch_set_tuning")

    def autotune_cached(self, A, key, path=None):
        """Panel widths for this batch from the JSON cache at `path` (default
        ~/.cache/paper_1406_5802_amd/batch_tuning.json) under `key`; on a miss, run
        the library's autotuner and store its choice.  Returns (widths, from_cache)."""
        import json
        import os

        path = path or os.path.join(os.path.expanduser("~"), ".cache", "paper_1406_5802_amd",
                                    "batch_tuning.json")
        table = {}
        if os.path.exists(path):
            with open(path) as fh:
                table = json.load(fh)
        if key in table:
            self.set_tuning(table[key]["nb"])
            return table[key]["nb"], True
        nb, ms = self.autotune(A)
        table[key] = {"nb": nb, "ms_per_bucket": ms}
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
        return nb, False

    def autotune(self, A):
        rc, nb, ms = _rmge.rmge_batch_autotune(self._h, A.data_ptr(), _stream_handle(A.device))
        if rc:
            raise RMGEError(rc, "rmge_batch_autotune")
        return nb, ms

    def lu(self, index, n, device="cuda"):
        import torch

        LU = torch.empty((n, n), dtype=torch.float64, device=device)
        rc = _rmge.rmge_batch_factors_lu(self._h, index, LU.data_ptr(), n, _stream_handle(LU.device))
        if rc:
            raise RMGEError(rc, "rmge_batch_factors_lu")
        return LU

    def close(self):
        if getattr(self, "_h", None):
            _rmge.rmge_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


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


__all__ = ["factor", "Factors", "Batch", "multiplier_params", "precondition", "schur_update", "grad_A",
           "RMGEError", "lib", "NONE", "GAUSSIAN", "CIRCULANT", "TOEPLITZ", "UNITARY_CIRCULANT",
           "F64", "F32", "BF16", "F32_BF16X2", "PIVOT_NONE", "PIVOT_BLOCK"]
