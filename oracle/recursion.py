"""The inverse BFGS matrix of eq. (3) applied to a block (oracle, test
infrastructure only).

apply_hk(h0, S, Y, V) returns B_k V, where B_k is built from B_0 = diag(h0) by the
pairs (s_i, y_i) in push order through eq. (3); with subtract_b0=True it returns
(B_k - B_0) V, the difference the probing of Alg. 2 and the randomized SVD of
Alg. 3 sample.  ``recursion.c`` evaluates eq. (3) as a recursion on the pair
index, one vector at a time (float64, OpenMP over columns); B_k is never formed.

Arrays use the (ncols, n) convention: row j of V is column j of the block.

Pinned by: hand-derived exact matrices (tests/golden), exact rationals, equality
with the dense eq. (3) matrix, the secant condition, symmetry, quadratic
termination, and planted mistakes that must fail those pins.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.ensure_built()
        L = ctypes.CDLL(path)
        L.oracle_apply_hk.restype = ctypes.c_int
        L.oracle_apply_hk.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                      ctypes.c_int32]
        L.oracle_max_threads.restype = ctypes.c_int
        L.oracle_philox4x64_10.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.oracle_normal_entry.restype = ctypes.c_double
        L.oracle_normal_entry.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64]
        L.oracle_normal_block.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                                          ctypes.c_void_p]
        _lib = L
    return _lib


def _c64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def apply_hk(h0, S, Y, V, subtract_b0: bool = False, nthreads: int = 0) -> np.ndarray:
    h0, S, Y, V = _c64(h0), _c64(S), _c64(Y), _c64(V)
    single = V.ndim == 1
    if single:
        V = V[None, :]
    n = h0.shape[0]
    k = S.shape[0] if S.size else 0
    if k:
        assert S.shape == (k, n) and Y.shape == (k, n)
    assert V.shape[1] == n
    out = np.empty_like(V)
    rc = lib().oracle_apply_hk(n, k, V.shape[0], h0.ctypes.data, S.ctypes.data if k else None,
                               Y.ctypes.data if k else None, V.ctypes.data, out.ctypes.data,
                               1 if subtract_b0 else 0, int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_apply_hk failed ({rc}): y_i^T s_i == 0")
    return out[0] if single else out


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def timed_apply_hk(h0, S, Y, V, nthreads: int = 0):
    t0 = time.perf_counter()
    out = apply_hk(h0, S, Y, V, nthreads=nthreads)
    return out, time.perf_counter() - t0
