"""O1: classical binary64 product (test infrastructure; see oracle/__init__.py).

The arithmetic lives in ``classical.c`` (the definition C_ij = sum_p A_ip B_pj,
Section 2.1 and Equation (1)); this module only marshals numpy arrays.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(path)
        i64 = ctypes.c_int64
        dp = ctypes.c_void_p
        lib.oracle_gemm_f64.argtypes = [i64, i64, i64, dp, i64, dp, i64, dp, i64]
        lib.oracle_gemm_f64.restype = None
        lib.oracle_gemm_rows_f64.argtypes = [i64, dp, i64, i64, dp, i64, dp, i64, dp, i64]
        lib.oracle_gemm_rows_f64.restype = None
        lib.oracle_gemm_rows_dot2_f64.argtypes = [i64, dp, i64, i64, dp, i64, dp, i64, dp, i64]
        lib.oracle_gemm_rows_dot2_f64.restype = None
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _as_f64(X):
    X = np.asarray(X)
    if X.dtype != np.float64:
        X = X.astype(np.float64)  # float32 widens exactly
    if not X.flags.c_contiguous:
        X = np.ascontiguousarray(X)
    return X


def gemm(A, B):
    """C = A @ B in binary64 with the i-p-j loop (ascending p)."""
    A = _as_f64(A)
    B = _as_f64(B)
    m, k = A.shape
    k2, n = B.shape
    assert k == k2
    C = np.empty((m, n), dtype=np.float64)
    if m and n:
        _lib().oracle_gemm_f64(m, k, n, A.ctypes.data, k, B.ctypes.data, n, C.ctypes.data, n)
    return C


def gemm_rows(A, B, rows, compensated=False):
    """Rows ``rows`` of A @ B (plain or Dot2-compensated)."""
    A = _as_f64(A)
    B = _as_f64(B)
    m, k = A.shape
    k2, n = B.shape
    assert k == k2
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    assert rows.size == 0 or (rows.min() >= 0 and rows.max() < m)
    out = np.empty((rows.size, n), dtype=np.float64)
    if rows.size and n:
        fn = _lib().oracle_gemm_rows_dot2_f64 if compensated else _lib().oracle_gemm_rows_f64
        fn(rows.size, rows.ctypes.data, k, n, A.ctypes.data, k, B.ctypes.data, n, out.ctypes.data, n)
    return out


def num_threads():
    return int(_lib().oracle_num_threads())


def gemm_exact(A, B):
    """Brute-force product for object (Fraction/int) arrays: the textbook
    definition with Python arithmetic, used on tiny inputs only."""
    m, k = len(A), len(A[0]) if len(A) else 0
    n = len(B[0]) if len(B) else 0
    return [[sum((A[i][p] * B[p][j] for p in range(k)), 0) for j in range(n)] for i in range(m)]
