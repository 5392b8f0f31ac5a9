"""Seeded input generator for the H^2 matrix-vector product.

Everything here produces inputs: seeded points and vectors, the serialized H^2
representation of a kernel matrix (built by ``builder.cpp``), and tiny random
representations for exactness tests.  It holds none of the matrix-vector
arithmetic, so both the oracle tests and the GPU library can consume its
output without sharing code with each other.
"""
from __future__ import annotations

import ctypes
import os
import weakref

import numpy as np

from . import fmt
from .randrep import random_rep  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libh2gen.so")

KERNELS = {"exp": 1, "laplace": 2, "poly2": 3, "one": 4, "gauss": 5}

# Workloads (see the design notes for how each stands in for the paper's sets)
CONFIGS = {
    "c1_2d_4096": dict(n=4096, dim=2, leaf=64, p=4, eta=0.7, kernel="exp", param=0.1,
                       seed_pts=1001, seed_vec=2001, nv=(1,)),
    "c2_2d_1m": dict(n=1 << 20, dim=2, leaf=64, p=6, eta=0.7, kernel="exp", param=0.1,
                     seed_pts=1002, seed_vec=2002, nv=(1, 16, 64), precisions=("fp32",)),
    "c3_3d_512k": dict(n=1 << 19, dim=3, leaf=64, p=4, eta=0.7, kernel="laplace", param=0.0,
                       seed_pts=1003, seed_vec=2003, nv=(64,), precisions=("bf16", "fp32")),
}

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        lib.h2gen_build.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int,
            ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int64)]
        lib.h2gen_build.restype = ctypes.c_int
        lib.h2gen_free.argtypes = [ctypes.c_void_p]
        lib.h2gen_free.restype = None
        _lib = lib
    return _lib


def points(n: int, dim: int, seed: int) -> np.ndarray:
    """n points uniform in [0,1]^dim, point-major (n x dim), from PCG64(seed)."""
    return np.random.default_rng(seed).random((n, dim))


def vectors(n: int, nv: int, seed: int) -> np.ndarray:
    """n x nv standard normal multi-vector, column-major (each vector contiguous)."""
    return np.random.default_rng(seed).standard_normal((nv, n)).T


class _Memory:
    """The builder's allocation; freed when the last reference goes."""

    def __init__(self, ptr: int, lib):
        self.ptr = ptr
        self._fin = weakref.finalize(self, lib.h2gen_free, ctypes.c_void_p(ptr))


class H2Buffer:
    """A serialized representation in host memory (from the C++ builder).

    ``array`` is a uint8 view that keeps the allocation alive by itself, so it
    stays valid after the H2Buffer object is gone; the memory is released when
    the buffer and every view of it are gone."""

    def __init__(self, ptr: int, nbytes: int, lib):
        mem = _Memory(ptr, lib)
        carr = (ctypes.c_uint8 * nbytes).from_address(ptr)
        carr._owner = mem  # the view -> ctypes array -> owner chain keeps the memory alive
        self.ptr = ptr
        self.nbytes = nbytes
        self.array = np.ctypeslib.as_array(carr)

    def free(self):
        """Drop this object's reference (memory goes once no view remains)."""
        self.array = None


def build(pts: np.ndarray, leaf: int, p: int, eta: float, kernel: str = "exp",
          param: float = 0.1, store_points: bool = False) -> H2Buffer:
    """Serialized H^2 representation of the kernel matrix on ``pts``."""
    lib = _load()
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    n, dim = pts.shape
    out = ctypes.c_void_p()
    ln = ctypes.c_int64()
    rc = lib.h2gen_build(pts.ctypes.data, n, dim, leaf, p, eta, KERNELS[kernel], param,
                         1 if store_points else 0, ctypes.byref(out), ctypes.byref(ln))
    if rc != 0:
        raise RuntimeError(f"h2gen_build failed with code {rc}")
    return H2Buffer(out.value, ln.value, lib)


def build_config(name: str, store_points: bool = False, **override) -> H2Buffer:
    c = dict(CONFIGS[name]); c.update(override)
    pts = points(c["n"], c["dim"], c["seed_pts"])
    return build(pts, c["leaf"], c["p"], c["eta"], c["kernel"], c["param"], store_points)
