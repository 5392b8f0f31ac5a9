"""CPU FP64 oracle of the H^2 matrix-vector product -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``h2_oracle.c`` (plain loops,
its own reader of the serialized representation) and shares no code with the
GPU library.  See the header of ``h2_oracle.c`` for what is computed.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libh2oracle.so")

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i64, dbl, ch, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_char, ctypes.c_int
        lib.h2o_open.argtypes = [vp, i64, ctypes.POINTER(vp)]
        lib.h2o_open.restype = ci
        lib.h2o_close.argtypes = [vp]
        lib.h2o_close.restype = None
        lib.h2o_n.argtypes = [vp]
        lib.h2o_n.restype = i64
        lib.h2o_gemv.argtypes = [vp, ch, dbl, vp, i64, i64, dbl, vp, i64, ci]
        lib.h2o_gemv.restype = ci
        lib.h2o_gemv_rows.argtypes = [vp, ch, dbl, vp, i64, i64, dbl, vp, i64, vp, i64, vp, ci]
        lib.h2o_gemv_rows.restype = ci
        lib.h2o_threads.argtypes = []
        lib.h2o_threads.restype = ci
        lib.h2o_set_threads.argtypes = [ci]
        lib.h2o_set_threads.restype = None
        lib.h2o_dense.argtypes = [vp, ch, vp]
        lib.h2o_dense.restype = ci
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    pass


def _fcol(a, n):
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a.reshape(n, 1)
    return np.asfortranarray(a)


class Oracle:
    """The reference product for one serialized representation (uint8 buffer)."""

    def __init__(self, buf: np.ndarray):
        lib = _load()
        self._buf = np.ascontiguousarray(np.asarray(buf).view(np.uint8).ravel())
        h = ctypes.c_void_p()
        rc = lib.h2o_open(self._buf.ctypes.data, self._buf.size, ctypes.byref(h))
        if rc != 0:
            raise OracleError(f"h2o_open failed ({rc})")
        self._h = h
        self.n = int(lib.h2o_n(h))

    def close(self):
        if self._h:
            _load().h2o_close(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def gemv(self, X, op="N", alpha=1.0, beta=0.0, Y=None, absval=False):
        """alpha op(A) X + beta Y (Y is not modified; a new array is returned)."""
        X = _fcol(X, self.n)
        nv = X.shape[1]
        Yo = np.zeros((self.n, nv), order="F") if Y is None else _fcol(Y, self.n).copy(order="F")
        rc = _load().h2o_gemv(self._h, op.encode(), alpha, X.ctypes.data, self.n, nv, beta,
                              Yo.ctypes.data, self.n, 1 if absval else 0)
        if rc != 0:
            raise OracleError(f"h2o_gemv failed ({rc})")
        return Yo

    def gemv_rows(self, rows, X, op="N", alpha=1.0, beta=0.0, Y=None, absval=False):
        """Rows ``rows`` (original indices) of alpha op(A) X + beta Y."""
        X = _fcol(X, self.n)
        nv = X.shape[1]
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        out = np.zeros((rows.size, nv), order="F")
        Y0 = None if Y is None else _fcol(Y, self.n)
        rc = _load().h2o_gemv_rows(self._h, op.encode(), alpha, X.ctypes.data, self.n, nv, beta,
                                   None if Y0 is None else Y0.ctypes.data, self.n,
                                   rows.ctypes.data, rows.size, out.ctypes.data, 1 if absval else 0)
        if rc != 0:
            raise OracleError(f"h2o_gemv_rows failed ({rc})")
        return out

    def dense(self, op="N"):
        """op(A) as an explicit n x n array (small n only)."""
        A = np.zeros((self.n, self.n), order="F")
        rc = _load().h2o_dense(self._h, op.encode(), A.ctypes.data)
        if rc != 0:
            raise OracleError(f"h2o_dense failed ({rc})")
        return A


def threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(_load().h2o_threads())


def set_threads(t: int) -> None:
    """Threads for the oracle's later OpenMP loops."""
    _load().h2o_set_threads(int(t))


def open_rep(buf) -> Oracle:
    return Oracle(buf)


def try_open(buf) -> int:
    """Return code of the oracle's reader on ``buf`` (0 = valid)."""
    lib = _load()
    b = np.ascontiguousarray(np.asarray(buf).view(np.uint8).ravel())
    h = ctypes.c_void_p()
    rc = lib.h2o_open(b.ctypes.data, b.size, ctypes.byref(h))
    if rc == 0:
        lib.h2o_close(h)
    return rc
