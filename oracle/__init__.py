"""FP64 CPU oracle for random-multiplier GENP -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  It is independent of the GPU library: it loads its
own C shared object (``rmge_oracle.c``) built with gcc, and never loads or
calls anything from the GPU package.

Each wrapper below cites the passage of Pan, Qian and Yan (arXiv:1406.5802)
that the underlying C function follows; the C file holds the arithmetic.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rmge_oracle.c")
_LIB = os.path.join(_HERE, "librmge_oracle.so")

NONE, GAUSSIAN, CIRCULANT, TOEPLITZ, UNITARY_CIRCULANT = 0, 1, 2, 3, 4
OK, ZERO_PIVOT, NONFINITE = 0, 4, 5


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP).  Returns the library path."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11",
           "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        i64, u64, i32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int
        dp = ctypes.POINTER(ctypes.c_double)
        vp = ctypes.c_void_p
        L.orc_philox4x64_10.argtypes = [vp, vp, vp]
        L.orc_words.argtypes = [u64, u64, i64, vp]
        L.orc_uniforms.argtypes = [u64, u64, i64, vp]
        L.orc_normals.argtypes = [u64, u64, i64, vp]
        L.orc_param_count.argtypes = [i32, i64]
        L.orc_param_count.restype = i64
        L.orc_multiplier_params.argtypes = [i32, i64, u64, vp]
        L.orc_multiplier_dense.argtypes = [i32, i64, vp, vp]
        L.orc_unitary_spectrum.argtypes = [i64, u64, vp, vp]
        L.orc_unitary_column.argtypes = [i64, vp, vp, vp, dp]
        L.orc_matmul.argtypes = [i64, i64, i64, vp, vp, vp]
        L.orc_genp.argtypes = [i64, vp, ctypes.POINTER(i64)]
        L.orc_genp_local.argtypes = [i64, i64, vp, vp, vp, ctypes.POINTER(i64)]
        L.orc_factor.argtypes = [i64, vp, i32, u64, vp, vp, vp]
        L.orc_factor_ex.argtypes = [i64, vp, i32, u64, i64, vp, vp, vp, vp, vp]
        L.orc_solve.argtypes = [i64, i64, vp, vp, vp, vp, vp, vp, i32, vp]
        L.orc_solve_adjoint.argtypes = [i64, i64, vp, vp, vp, vp, vp]
        L.orc_errors.argtypes = [i64, i64, vp, vp, vp, dp, dp]
        L.orc_grad_A.argtypes = [i64, i64, vp, vp, vp]
        L.orc_num_threads.restype = i32
        L.orc_set_num_threads.argtypes = [i32]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class _Stats(ctypes.Structure):
    _fields_ = [("info", ctypes.c_int64), ("status", ctypes.c_int32),
                ("steps", ctypes.c_int32), ("eta", ctypes.c_double * 17),
                ("relres", ctypes.c_double * 17), ("min_abs_pivot", ctypes.c_double),
                ("growth", ctypes.c_double)]


# --------------------------------------------------------------------------
# Random numbers (Philox4x64-10, SC'11; Box-Muller normals; Definition defrndm)
# --------------------------------------------------------------------------

def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint64).copy()
    k = np.asarray(key, dtype=np.uint64).copy()
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_p(c), _p(k), _p(out))
    return out


def words(seed: int, stream: int, nblocks: int) -> np.ndarray:
    out = np.zeros(4 * nblocks, dtype=np.uint64)
    lib().orc_words(seed, stream, nblocks, _p(out))
    return out


def uniforms(seed: int, stream: int, count: int) -> np.ndarray:
    out = np.zeros(count, dtype=np.float64)
    lib().orc_uniforms(seed, stream, count, _p(out))
    return out


def normals(seed: int, stream: int, count: int) -> np.ndarray:
    out = np.zeros(count, dtype=np.float64)
    lib().orc_normals(seed, stream, count, _p(out))
    return out


# --------------------------------------------------------------------------
# Multipliers (Definition defrndm; Section 6 circulant; Toeplitz blocks)
# --------------------------------------------------------------------------

def param_count(kind: int, n: int) -> int:
    return int(lib().orc_param_count(kind, n))


def multiplier_params(kind: int, n: int, seed: int) -> np.ndarray:
    out = np.zeros(param_count(kind, n), dtype=np.float64)
    if out.size:
        lib().orc_multiplier_params(kind, n, seed, _p(out))
    return out


def unitary_spectrum(n: int, seed: int) -> np.ndarray:
    """The unit-modulus, conjugate-symmetric spectrum u of the random unitary
    circulant (Section 6, Example exunc, step (i)), as complex values."""
    re = np.zeros(n, dtype=np.float64)
    im = np.zeros(n, dtype=np.float64)
    lib().orc_unitary_spectrum(n, seed, _p(re), _p(im))
    return re + 1j * im


def unitary_column(u) -> tuple[np.ndarray, float]:
    """c = Omega^{-1} u by the plain O(n^2) sum (Example exunc, step (ii));
    returns c and the largest imaginary part that cancelled."""
    u = np.asarray(u, dtype=np.complex128)
    re, im = _f64(u.real), _f64(u.imag)
    c = np.zeros(u.size, dtype=np.float64)
    worst = ctypes.c_double(0.0)
    lib().orc_unitary_column(u.size, _p(re), _p(im), _p(c), ctypes.byref(worst))
    return c, float(worst.value)


def multiplier_dense(kind: int, n: int, params=None) -> np.ndarray:
    H = np.zeros((n, n), dtype=np.float64)
    p = _f64(params) if params is not None else np.zeros(1)
    rc = lib().orc_multiplier_dense(kind, n, _p(p), _p(H))
    if rc:
        raise ValueError("bad multiplier kind %r" % kind)
    return H


def multiplier(kind: int, n: int, seed: int) -> np.ndarray:
    """Dense H drawn from ``seed`` (identity for NONE)."""
    if kind == NONE:
        return multiplier_dense(NONE, n)
    return multiplier_dense(kind, n, multiplier_params(kind, n, seed))


def matmul(A, B) -> np.ndarray:
    A, B = _f64(A), _f64(B)
    m, q = A.shape
    q2, p = B.shape
    assert q == q2
    C = np.zeros((m, p), dtype=np.float64)
    lib().orc_matmul(m, q, p, _p(A), _p(B), _p(C))
    return C


# --------------------------------------------------------------------------
# GENP (Section 3, eq. eqgenp with unit pivot blocks; Corollary corec)
# --------------------------------------------------------------------------

def genp(M) -> tuple[np.ndarray, int, int]:
    """Unpivoted LU of M in place on a copy; returns (LU, status, info)."""
    LU = _f64(M).copy()
    info = ctypes.c_int64(-1)
    rc = lib().orc_genp(LU.shape[0], _p(LU), ctypes.byref(info))
    return LU, int(rc), int(info.value)


def _ends(blocks, n: int) -> np.ndarray:
    """Block ends as int64, checked to partition 0..n."""
    e = np.asarray(list(blocks), dtype=np.int64)
    if e.size == 0 or e[-1] != n or np.any(np.diff(np.concatenate([[0], e])) <= 0):
        raise ValueError("pivot blocks must be strictly increasing ends reaching n=%d" % n)
    return e


def genp_local(M, blocks) -> tuple[np.ndarray, np.ndarray, int, int]:
    """Block elimination whose recursion (eq. eqgenp) stops at the given diagonal
    blocks, each eliminated with partial pivoting confined to the block (Section 3,
    after eq. eqgenpin: small blocks go to a black-box method).  ``blocks`` lists
    the blocks' ends (strictly increasing, the last = n): the caller chooses the
    partition.  Returns (LU, perm, status, info) with (P M)[t] = M[perm[t]] =
    (L U)[t]."""
    LU = _f64(M).copy()
    n = LU.shape[0]
    ends = _ends(blocks, n)
    perm = np.zeros(n, dtype=np.int64)
    info = ctypes.c_int64(-1)
    rc = lib().orc_genp_local(n, len(ends), _p(ends), _p(LU), _p(perm), ctypes.byref(info))
    return LU, perm, int(rc), int(info.value)


def uniform_blocks(n: int, w: int) -> list:
    """Ends of consecutive diagonal blocks of width w (the last may be narrower)."""
    return list(range(w, n, w)) + [n]


@dataclass
class Factors:
    n: int
    kind: int
    seed: int
    A: np.ndarray
    H: np.ndarray
    LU: np.ndarray
    status: int
    info: int
    min_abs_pivot: float
    growth: float
    seconds: float = 0.0
    perm: np.ndarray | None = None  # row order of P M = L U (None: no pivoting)
    pivot_blocks: tuple = ()        # ends of the pivoting blocks (empty: no pivoting)


@dataclass
class Solution:
    X: np.ndarray
    eta: list = field(default_factory=list)
    relres: list = field(default_factory=list)
    seconds: float = 0.0


def factor(A, kind: int, seed: int, pivot_blocks=None) -> Factors:
    """M = A H (Fact faprepr), then GENP on M; with ``pivot_blocks`` (the ends of
    the diagonal blocks), the locally pivoted block elimination of
    :func:`genp_local` instead."""
    A = _f64(A)
    n = A.shape[0]
    H = np.zeros((n, n))
    LU = np.zeros((n, n))
    ends = _ends(pivot_blocks, n) if pivot_blocks is not None else None
    perm = np.zeros(n, dtype=np.int64) if ends is not None else None
    st = _Stats()
    t0 = time.perf_counter()
    rc = lib().orc_factor_ex(n, _p(A), kind, seed, 0 if ends is None else len(ends),
                             _p(ends) if ends is not None else None, _p(H), _p(LU),
                             _p(perm) if perm is not None else None, ctypes.byref(st))
    dt = time.perf_counter() - t0
    return Factors(n, kind, seed, A, H, LU, int(rc), int(st.info),
                   float(st.min_abs_pivot), float(st.growth), dt, perm,
                   tuple(int(e) for e in ends) if ends is not None else ())


def _perm(f: Factors):
    return _p(f.perm) if f.perm is not None else None


def solve(f: Factors, B, refine: int = 1) -> Solution:
    """x = H (LU)^{-1} b, then ``refine`` FP64 refinement steps (Section 8.1)."""
    B = _f64(B)
    vec = B.ndim == 1
    if vec:
        B = B[:, None]
    nrhs = B.shape[1]
    X = np.zeros_like(B)
    st = _Stats()
    t0 = time.perf_counter()
    lib().orc_solve(f.n, nrhs, _p(f.A), _p(f.H), _p(f.LU), _perm(f), _p(B), _p(X), refine,
                    ctypes.byref(st))
    dt = time.perf_counter() - t0
    X = X[:, 0] if vec else X
    return Solution(X, [st.eta[i] for i in range(refine + 1)],
                    [st.relres[i] for i in range(refine + 1)], dt)


def solve_adjoint(f: Factors, W) -> np.ndarray:
    """Y = A^{-T} W = P^T L^{-T} U^{-T} H^T W."""
    W = _f64(W)
    vec = W.ndim == 1
    if vec:
        W = W[:, None]
    Y = np.zeros_like(W)
    lib().orc_solve_adjoint(f.n, W.shape[1], _p(f.H), _p(f.LU), _perm(f), _p(W), _p(Y))
    return Y[:, 0] if vec else Y


def errors(A, B, X) -> tuple[float, float]:
    """(eta_inf, relres_2) on the original A, max over right-hand sides."""
    A, B, X = _f64(A), _f64(B), _f64(X)
    if B.ndim == 1:
        B, X = B[:, None], X[:, None]
    e, r = ctypes.c_double(), ctypes.c_double()
    lib().orc_errors(A.shape[0], B.shape[1], _p(A), _p(B), _p(X), ctypes.byref(e),
                     ctypes.byref(r))
    return e.value, r.value


def grad_A(gb, X) -> np.ndarray:
    gb, X = _f64(gb), _f64(X)
    if gb.ndim == 1:
        gb, X = gb[:, None], X[:, None]
    n = gb.shape[0]
    G = np.zeros((n, n))
    lib().orc_grad_A(n, gb.shape[1], _p(gb), _p(X), _p(G))
    return G


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(t: int) -> None:
    """Threads the row loops use (results do not depend on it)."""
    lib().orc_set_num_threads(int(t))
