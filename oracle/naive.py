"""The naive method, c_ij = sum_{p} a_ip * b_pj (Section 2.1, Algorithm 1).

Test infrastructure only.  Two independent writings of the same definition:

* ``gemm``      the C triple loop of ``gemm_f64.c`` in IEEE double, loop order
                i-p-j, summation over p in increasing order, no fused
                multiply-add; OpenMP over rows (thread count does not change
                a single bit of the result).
* ``naive_py``  Algorithm 1 as printed (i, j, then the running sum over p) in
                plain Python.  On Python ``int`` entries it is exact, which is
                what the integer checks rely on.  Use it for tiny inputs only.

Dimensions follow the cutoff section's naming: A is m x k, B is k x n.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        lib.oracle_gemm_f64.restype = ctypes.c_int
        lib.oracle_gemm_f64.argtypes = [
            ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int]
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def gemm(A, B, threads: int = 0) -> np.ndarray:
    """C = A @ B in double precision by the triple loop.

    ``A`` (m x k) and ``B`` (k x n) may be any real dtype; they are converted
    to float64 first (exact for float32 and for integers below 2**53).
    """
    A = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
    B = np.ascontiguousarray(np.asarray(B, dtype=np.float64))
    if A.ndim != 2 or B.ndim != 2 or A.shape[1] != B.shape[0]:
        raise ValueError(f"shape mismatch {A.shape} x {B.shape}")
    m, k = A.shape
    n = B.shape[1]
    C = np.empty((m, n), dtype=np.float64)
    rc = _load().oracle_gemm_f64(m, n, k,
                                 A.ctypes.data, max(k, 1),
                                 B.ctypes.data, max(n, 1),
                                 C.ctypes.data, max(n, 1), int(threads))
    if rc != 0:
        raise ValueError("oracle_gemm_f64 rejected its arguments")
    return C


def gemm_rows(A, B, rows, threads: int = 0) -> np.ndarray:
    """Rows ``rows`` of A @ B, each computed exactly as ``gemm`` would.

    Row i of the product depends only on row i of A, so this is the full
    oracle restricted to a sample of outputs (used at sizes where the whole
    triple loop would take too long on the host).
    """
    rows = np.asarray(rows, dtype=np.int64)
    return gemm(np.asarray(A)[rows, :], B, threads=threads)


def naive_py(A, B):
    """Algorithm 1 literally, on nested Python lists (exact for ints)."""
    A = [list(r) for r in A]
    B = [list(r) for r in B]
    m = len(A)
    k = len(B)
    n = len(B[0]) if k else 0
    if any(len(r) != k for r in A):
        raise ValueError("shape mismatch")
    C = [[0] * n for _ in range(m)]
    for i in range(m):
        for j in range(n):
            soma = 0
            for p in range(k):
                soma = soma + A[i][p] * B[p][j]
            C[i][j] = soma
    return C
