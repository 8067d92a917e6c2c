"""Differentiable solve X = A^{-1} B through the random-multiplier factorization.

Forward: factor A H = (P^T) L U on the GPU and solve, refined in FP64 to a backward
error tol (classical refinement for FP64 factors, GMRES-based refinement for FP32
factors).  Backward, by hand (differentiating A X = B; the multiplier cancels since
A^{-1} = H (A H)^{-1}, Fact faprepr):

    grad_B = A^{-T} grad_X          (the adjoint solve, reusing L, U and H, refined)
    grad_A = -grad_B X^T            (rmge_grad_A)

Every step runs in the library's kernels; PyTorch supplies memory and the stream.
"""
from __future__ import annotations

import torch

from . import _rmge
from ._rmge import RMGEError


# Factorization handles of finished solves, kept for reuse by the next solve of
# the same shape and options: a handle owns its n x n factors and workspaces,
# and allocating and freeing them costs about as much as the factorization
# itself at n = 8192 (rmge_refactor reuses them).  A handle is in this list only
# while no solve holds it.
_free: dict = {}
_MAX_FREE = 2


def _key(A, kind, block, prec, pivot):
    return (A.shape[0], A.device.index, kind, block, prec, pivot)


def _acquire(A, kind, seed, block, prec, pivot):
    from . import Factors

    idle = _free.get(_key(A, kind, block, prec, pivot))
    if idle:
        f = idle.pop()
        f.refactor(A, seed=seed)
        return f
    return Factors(A, kind=kind, seed=seed, block=block, prec=prec, pivot=pivot)


def _release(f, key):
    f.A = None  # the handle no longer keeps the caller's matrix alive
    idle = _free.setdefault(key, [])
    if len(idle) < _MAX_FREE:
        idle.append(f)
    else:
        f.close()


class RmgeSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, B, kind, seed, block, prec, pivot, tol, max_iters):
        from . import F32, F32_BF16X2

        A = A.detach().contiguous()
        B = B.detach().contiguous()
        key = _key(A, kind, block, prec, pivot)
        f = _acquire(A, kind, seed, block, prec, pivot)
        if not f.ok:
            status = f.status
            _release(f, key)
            raise RMGEError(status, "RmgeSolve.forward (factor)")
        if prec in (F32, F32_BF16X2):
            X, st = f.solve_gmres(B, max_iters=max_iters, restart=32, tol=tol)
        else:
            X, st = f.solve(B, max_refine=16, tol=tol)
        if not st["converged"]:
            _release(f, key)
            raise RMGEError(_rmge.RMGE_NOT_CONVERGED, "RmgeSolve.forward (solve)")
        ctx.f, ctx.key = f, key
        ctx.prec, ctx.tol, ctx.max_iters = prec, tol, max_iters
        ctx.save_for_backward(X)
        return X

    @staticmethod
    def backward(ctx, gX):
        from . import F32, F32_BF16X2

        f = ctx.f
        (X,) = ctx.saved_tensors
        gX = gX.contiguous()
        if ctx.prec in (F32, F32_BF16X2):
            GB, st = f.solve_gmres(gX, max_iters=ctx.max_iters, restart=32, tol=ctx.tol,
                                   trans=True)
        else:
            GB, st = f.solve_adjoint_refined(gX, max_refine=16, tol=ctx.tol)
        if not st["converged"]:
            _release(f, ctx.key)
            ctx.f = None
            raise RMGEError(_rmge.RMGE_NOT_CONVERGED, "RmgeSolve.backward (adjoint)")
        grad_A = None
        if ctx.needs_input_grad[0]:
            n, nrhs = X.shape
            grad_A = torch.empty((n, n), dtype=torch.float64, device=X.device)
            rc = _rmge.rmge_grad_A(GB.data_ptr(), GB.stride(0), X.data_ptr(), X.stride(0), n,
                                   nrhs, grad_A.data_ptr(), grad_A.stride(0),
                                   int(torch.cuda.current_stream(X.device).cuda_stream))
            if rc:
                raise RMGEError(rc, "rmge_grad_A")
        grad_B = GB if ctx.needs_input_grad[1] else None
        _release(f, ctx.key)
        ctx.f = None
        return grad_A, grad_B, None, None, None, None, None, None, None


def solve(A, B, kind=None, seed=0, block=256, prec=None, pivot=None, tol=1e-14, max_iters=400):
    """X = A^{-1} B, differentiable in A and B.  A: n x n, B: n or n x nrhs (nrhs <= 64),
    float64 CUDA tensors.  kind, prec, pivot as for factor()."""
    from . import F64, GAUSSIAN, PIVOT_NONE, _kind

    kind = GAUSSIAN if kind is None else _kind(kind)
    prec = F64 if prec is None else prec
    pivot = PIVOT_NONE if pivot is None else pivot
    vec = B.dim() == 1
    B2 = B.reshape(-1, 1) if vec else B
    X = RmgeSolve.apply(A, B2, kind, seed, block, prec, pivot, tol, max_iters)
    return X.reshape(-1) if vec else X
