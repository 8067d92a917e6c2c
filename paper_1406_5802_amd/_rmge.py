"""ctypes declarations of the C ABI in include/rmge.h (same names, same arguments).

Loading fails loudly if ``librmge.so`` has not been built: there is no CPU
fallback for any step of the method.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librmge.so")

(RMGE_MULT_NONE, RMGE_MULT_GAUSSIAN, RMGE_MULT_CIRCULANT, RMGE_MULT_TOEPLITZ,
 RMGE_MULT_UNITARY_CIRCULANT) = 0, 1, 2, 3, 4
RMGE_F64, RMGE_F32, RMGE_BF16, RMGE_F32_BF16X2 = 0, 1, 2, 3
RMGE_PIVOT_NONE, RMGE_PIVOT_BLOCK = 0, 1
(RMGE_OK, RMGE_EINVAL, RMGE_ENOMEM, RMGE_EDEVICE, RMGE_ZERO_PIVOT, RMGE_NONFINITE,
 RMGE_NOT_CONVERGED) = range(7)

STATUS_NAMES = {
    0: "RMGE_OK", 1: "RMGE_EINVAL", 2: "RMGE_ENOMEM", 3: "RMGE_EDEVICE",
    4: "RMGE_ZERO_PIVOT", 5: "RMGE_NONFINITE", 6: "RMGE_NOT_CONVERGED",
}

# Every function the header declares, for the export check.
EXPORTS = (
    "rmge_factor", "rmge_factor_ex", "rmge_factor_pivoted", "rmge_refactor", "rmge_solve",
    "rmge_solve_gmres", "rmge_solve_adjoint", "rmge_solve_adjoint_ex", "rmge_grad_A",
    "rmge_factor_stats_get", "rmge_factor_times", "rmge_factor_update_time", "rmge_factors_lu",
    "rmge_factors_perm", "rmge_multiplier_params", "rmge_param_count", "rmge_precondition",
    "rmge_precondition_noalloc", "rmge_schur_update_f32", "rmge_batch_create", "rmge_batch_run",
    "rmge_batch_run_timed", "rmge_batch_graph_run", "rmge_batch_results", "rmge_batch_get_tuning",
    "rmge_batch_set_tuning", "rmge_batch_autotune", "rmge_batch_factors_lu", "rmge_batch_destroy",
    "rmge_destroy", "rmge_status_string", "rmge_version",
)


class rmge_factor_stats(ctypes.Structure):
    _fields_ = [("info", ctypes.c_int64), ("status", ctypes.c_int32), ("block", ctypes.c_int32),
                ("min_abs_pivot", ctypes.c_double), ("growth", ctypes.c_double),
                ("ms_multiplier", ctypes.c_double), ("ms_product", ctypes.c_double),
                ("ms_factor", ctypes.c_double)]


RMGE_BATCH_BUCKETS = 5


class rmge_batch_system(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("kind", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("a_off", ctypes.c_int64), ("v_off", ctypes.c_int64)]


class rmge_batch_tuning(ctypes.Structure):
    _fields_ = [("nb", ctypes.c_int32 * RMGE_BATCH_BUCKETS)]


class rmge_solve_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("eta0", ctypes.c_double), ("eta", ctypes.c_double),
                ("eta_hist", ctypes.c_double * 17)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it was never built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            "librmge.so is not built (expected %s); build it with "
            "`python paper_1406_5802_amd/build.py` -- there is no fallback" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    i64, i32, u64, vp, dp = (ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_void_p,
                             ctypes.c_void_p)
    hp = ctypes.POINTER(ctypes.c_void_p)
    L.rmge_factor.argtypes = [dp, i64, i32, u64, i32, hp]
    L.rmge_factor_ex.argtypes = [dp, i64, i64, i32, u64, i32, i32, vp, hp]
    L.rmge_factor_pivoted.argtypes = [dp, i64, i64, i32, u64, i32, i32, i32, vp, hp]
    L.rmge_factors_perm.argtypes = [vp, vp]
    L.rmge_grad_A.argtypes = [dp, i64, dp, i64, i64, i64, dp, i64, vp]
    L.rmge_refactor.argtypes = [vp, dp, i64, u64]
    L.rmge_solve.argtypes = [vp, dp, i64, i64, dp, i64, i32, ctypes.c_double,
                             ctypes.POINTER(rmge_solve_stats)]
    L.rmge_solve_gmres.argtypes = [vp, i32, dp, i64, i64, dp, i64, i32, i32, ctypes.c_double,
                                   ctypes.POINTER(rmge_solve_stats)]
    L.rmge_solve_adjoint.argtypes = [vp, dp, i64, i64, dp, i64]
    L.rmge_solve_adjoint_ex.argtypes = [vp, dp, i64, i64, dp, i64, i32, ctypes.c_double,
                                        ctypes.POINTER(rmge_solve_stats)]
    L.rmge_factor_stats_get.argtypes = [vp, ctypes.POINTER(rmge_factor_stats)]
    L.rmge_factor_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.rmge_factor_update_time.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double)]
    L.rmge_factors_lu.argtypes = [vp, dp, i64]
    L.rmge_multiplier_params.argtypes = [i32, i64, u64, dp, vp]
    L.rmge_param_count.argtypes = [i32, i64]
    L.rmge_param_count.restype = i64
    L.rmge_precondition.argtypes = [dp, i64, i64, i32, u64, dp, i64, vp]
    L.rmge_precondition_noalloc.argtypes = [dp, i64, i64, i32, u64, dp, i64, vp]
    L.rmge_schur_update_f32.argtypes = [i64, i64, i64, dp, i64, dp, i64, dp, i64, i32, vp]
    bp = ctypes.POINTER(rmge_batch_tuning)
    L.rmge_batch_create.argtypes = [ctypes.POINTER(rmge_batch_system), i32, bp, i32, i32, hp]
    L.rmge_batch_run.argtypes = [vp, dp, dp, dp, ctypes.c_double, vp]
    L.rmge_batch_graph_run.argtypes = [vp, dp, dp, dp, ctypes.c_double, vp]
    L.rmge_batch_run_timed.argtypes = [vp, dp, dp, dp, ctypes.c_double, vp,
                                       ctypes.POINTER(ctypes.c_double)]
    L.rmge_batch_results.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.rmge_batch_get_tuning.argtypes = [vp, bp]
    L.rmge_batch_set_tuning.argtypes = [vp, bp]
    L.rmge_batch_autotune.argtypes = [vp, dp, vp, bp, vp]
    L.rmge_batch_factors_lu.argtypes = [vp, i32, dp, i64, vp]
    L.rmge_batch_destroy.argtypes = [vp]
    L.rmge_batch_destroy.restype = None
    L.rmge_destroy.argtypes = [vp]
    L.rmge_destroy.restype = None
    L.rmge_status_string.argtypes = [i32]
    L.rmge_status_string.restype = ctypes.c_char_p
    L.rmge_version.restype = i32
    for name in ("rmge_factor", "rmge_factor_ex", "rmge_factor_pivoted", "rmge_refactor",
                 "rmge_solve", "rmge_solve_gmres", "rmge_solve_adjoint", "rmge_solve_adjoint_ex",
                 "rmge_grad_A", "rmge_factor_stats_get", "rmge_factor_times",
                 "rmge_factor_update_time", "rmge_factors_lu",
                 "rmge_factors_perm",
                 "rmge_multiplier_params", "rmge_precondition", "rmge_precondition_noalloc",
                 "rmge_schur_update_f32", "rmge_batch_create", "rmge_batch_run",
                 "rmge_batch_run_timed",
                 "rmge_batch_graph_run", "rmge_batch_results", "rmge_batch_get_tuning",
                 "rmge_batch_set_tuning", "rmge_batch_autotune", "rmge_batch_factors_lu"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def status_string(s: int) -> str:
    return lib().rmge_status_string(int(s)).decode()


class RMGEError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = int(status)
        name = STATUS_NAMES.get(self.status, str(status))
        super().__init__("%s%s: %s" % (what + " -> " if what else "", name,
                                       status_string(self.status) if _lib else name))


# Thin wrappers with the C names: pointers are ints (device addresses).

def rmge_factor_ex(A: int, n: int, lda: int, kind: int, seed: int, block: int, prec: int,
                   stream: int):
    h = ctypes.c_void_p()
    rc = lib().rmge_factor_ex(A, n, lda, kind, ctypes.c_uint64(seed & (2**64 - 1)), block, prec,
                              stream, ctypes.byref(h))
    return rc, h


def rmge_factor_pivoted(A: int, n: int, lda: int, kind: int, seed: int, block: int, prec: int,
                        pivot: int, stream: int):
    h = ctypes.c_void_p()
    rc = lib().rmge_factor_pivoted(A, n, lda, kind, ctypes.c_uint64(seed & (2**64 - 1)), block,
                                   prec, pivot, stream, ctypes.byref(h))
    return rc, h


def rmge_factor(A: int, n: int, kind: int, seed: int, block: int):
    h = ctypes.c_void_p()
    rc = lib().rmge_factor(A, n, kind, ctypes.c_uint64(seed & (2**64 - 1)), block, ctypes.byref(h))
    return rc, h


def rmge_refactor(h, A: int, lda: int, seed: int) -> int:
    return lib().rmge_refactor(h, A, lda, ctypes.c_uint64(seed & (2**64 - 1)))


def rmge_solve(h, B: int, nrhs: int, ldb: int, X: int, ldx: int, max_refine: int, tol: float):
    st = rmge_solve_stats()
    rc = lib().rmge_solve(h, B, nrhs, ldb, X, ldx, max_refine, tol, ctypes.byref(st))
    return rc, st


def rmge_solve_gmres(h, trans: int, B: int, nrhs: int, ldb: int, X: int, ldx: int,
                     max_iters: int, restart: int, tol: float):
    st = rmge_solve_stats()
    rc = lib().rmge_solve_gmres(h, trans, B, nrhs, ldb, X, ldx, max_iters, restart, tol,
                                ctypes.byref(st))
    return rc, st


def rmge_solve_adjoint(h, W: int, nrhs: int, ldw: int, Y: int, ldy: int) -> int:
    return lib().rmge_solve_adjoint(h, W, nrhs, ldw, Y, ldy)


def rmge_solve_adjoint_ex(h, W: int, nrhs: int, ldw: int, Y: int, ldy: int, max_refine: int,
                          tol: float):
    st = rmge_solve_stats()
    rc = lib().rmge_solve_adjoint_ex(h, W, nrhs, ldw, Y, ldy, max_refine, tol, ctypes.byref(st))
    return rc, st


def rmge_grad_A(GB: int, ldgb: int, X: int, ldx: int, n: int, nrhs: int, GA: int, ldga: int,
                stream: int) -> int:
    return lib().rmge_grad_A(GB, ldgb, X, ldx, n, nrhs, GA, ldga, stream)


def rmge_factor_stats_get(h):
    st = rmge_factor_stats()
    rc = lib().rmge_factor_stats_get(h, ctypes.byref(st))
    return rc, st


def rmge_factor_times(h):
    ms = (ctypes.c_double * 3)()
    rc = lib().rmge_factor_times(h, ms)
    return rc, (ms[0], ms[1], ms[2])


def rmge_factor_update_time(h):
    ms, fl = ctypes.c_double(), ctypes.c_double()
    rc = lib().rmge_factor_update_time(h, ctypes.byref(ms), ctypes.byref(fl))
    return rc, ms.value, fl.value


def rmge_factors_lu(h, LU: int, ld: int) -> int:
    return lib().rmge_factors_lu(h, LU, ld)


def rmge_factors_perm(h, perm: int) -> int:
    return lib().rmge_factors_perm(h, perm)


def rmge_multiplier_params(kind: int, n: int, seed: int, out: int, stream: int) -> int:
    return lib().rmge_multiplier_params(kind, n, ctypes.c_uint64(seed & (2**64 - 1)), out, stream)


def rmge_param_count(kind: int, n: int) -> int:
    return int(lib().rmge_param_count(kind, n))


def rmge_precondition(A: int, n: int, lda: int, kind: int, seed: int, M: int, ldm: int,
                      stream: int) -> int:
    return lib().rmge_precondition(A, n, lda, kind, ctypes.c_uint64(seed & (2**64 - 1)), M, ldm,
                                   stream)


def rmge_destroy(h) -> None:
    lib().rmge_destroy(h)


def rmge_status_string(s: int) -> str:
    return status_string(s)


def rmge_version() -> int:
    return int(lib().rmge_version())


def rmge_precondition_noalloc(A: int, n: int, lda: int, kind: int, seed: int, M: int, ldm: int,
                              stream: int) -> int:
    return lib().rmge_precondition_noalloc(A, n, lda, kind, ctypes.c_uint64(seed & (2**64 - 1)),
                                           M, ldm, stream)


def rmge_schur_update_f32(M: int, N: int, K: int, D: int, ldd: int, E: int, lde: int, C: int,
                          ldc: int, terms: int, stream: int) -> int:
    return lib().rmge_schur_update_f32(M, N, K, D, ldd, E, lde, C, ldc, terms, stream)


def rmge_batch_create(systems, tuning, restart: int, max_iters: int):
    arr = (rmge_batch_system * len(systems))(*systems)
    h = ctypes.c_void_p()
    rc = lib().rmge_batch_create(arr, len(systems), ctypes.byref(tuning) if tuning else None,
                                 restart, max_iters, ctypes.byref(h))
    return rc, h


def rmge_batch_run(h, A: int, B: int, X: int, tol: float, stream: int) -> int:
    return lib().rmge_batch_run(h, A, B, X, tol, stream)


def rmge_batch_run_timed(h, A: int, B: int, X: int, tol: float, stream: int):
    ms = (ctypes.c_double * 4)()
    rc = lib().rmge_batch_run_timed(h, A, B, X, tol, stream, ms)
    return rc, (ms[0], ms[1], ms[2], ms[3])


def rmge_batch_graph_run(h, A: int, B: int, X: int, tol: float, stream: int) -> int:
    return lib().rmge_batch_graph_run(h, A, B, X, tol, stream)


def rmge_batch_results(h, status, eta, eta0, iters, info, fp64, stream: int) -> int:
    """Host numpy arrays (int32, float64, float64, int32, int64, int32) or None."""
    def ptr(a):
        return None if a is None else a.ctypes.data_as(ctypes.c_void_p)
    return lib().rmge_batch_results(h, ptr(status), ptr(eta), ptr(eta0), ptr(iters), ptr(info),
                                    ptr(fp64), stream)


def rmge_batch_get_tuning(h):
    t = rmge_batch_tuning()
    rc = lib().rmge_batch_get_tuning(h, ctypes.byref(t))
    return rc, list(t.nb)


def rmge_batch_set_tuning(h, nb) -> int:
    t = rmge_batch_tuning((ctypes.c_int32 * RMGE_BATCH_BUCKETS)(*nb))
    return lib().rmge_batch_set_tuning(h, ctypes.byref(t))


def rmge_batch_autotune(h, A: int, stream: int):
    t = rmge_batch_tuning()
    ms = (ctypes.c_double * RMGE_BATCH_BUCKETS)()
    rc = lib().rmge_batch_autotune(h, A, stream, ctypes.byref(t), ms)
    return rc, list(t.nb), list(ms)


def rmge_batch_factors_lu(h, index: int, LU: int, ld: int, stream: int) -> int:
    return lib().rmge_batch_factors_lu(h, index, LU, ld, stream)


def rmge_batch_destroy(h) -> None:
    lib().rmge_batch_destroy(h)
