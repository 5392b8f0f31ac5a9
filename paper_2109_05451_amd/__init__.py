"""MI355X H^2 matrix-vector product: Python binding of libh2gemv.so.

Argument marshalling only.  Every step of the product runs in the HIP
kernels of ``libh2gemv.so`` behind the C ABI of ``include/h2.h``; PyTorch is
used for device memory and streams.  There is no CPU fallback: if the library
is not built, importing works but constructing an operator raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libh2gemv.so")

H2_OK, H2_EINVAL, H2_EIO, H2_EFORMAT, H2_ENOMEM, H2_EHIP, H2_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6

# exported symbols of include/h2.h, in declaration order
EXPORTS = ("h2_load", "h2_load_mem", "h2_validate", "h2_gemv", "h2_gemv_ex", "h2_gemv_noalloc", "h2_graph", "h2_prepare", "h2_reserve", "h2_tune",
           "h2_compress", "h2_export", "h2_ranks", "h2_plan_info", "h2_tune_set", "h2_set_dense_grid", "h2_set_schedule",
           "h2_set_sweeps", "h2_set_fragment_order", "h2_stats", "h2_level_stats", "h2_n", "h2_profile", "h2_profile_read", "h2_free", "h2_batch_load", "h2_batch_load_ex", "h2_batch_gemv",
           "h2_batch_tune", "h2_batch_graph", "h2_batch_info", "h2_batch_plan_info", "h2_batch_free", "h2_server_create",
           "h2_server_submit", "h2_server_wait", "h2_server_stats", "h2_server_free", "h2_last_error")

PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2}


class H2Stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "n", "depth", "nnodes", "nleaves", "ncoupling", "ndense", "csp", "csp_dense",
        "entries_U", "entries_V", "entries_E", "entries_F", "entries_S", "entries_D",
        "tree_rows", "shared_basis", "device_bytes", "max_rank", "max_leaf")] + [
        (name, ctypes.c_double) for name in ("alg_flops_per_vector", "alg_bytes_matrix", "alg_bytes_per_vector")]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class H2LevelStats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "nodes", "krow", "kcol", "coupling_blocks", "csp", "entries_S", "entries_E", "entries_F")]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class H2CompressInfo(ctypes.Structure):
    _fields_ = [("ms_orthogonalize", ctypes.c_double), ("ms_reweight", ctypes.c_double),
                ("ms_truncate", ctypes.c_double), ("ms_project", ctypes.c_double),
                ("ms_assemble", ctypes.c_double), ("lowrank_entries_before", ctypes.c_int64),
                ("lowrank_entries_after", ctypes.c_int64), ("sigma_ref_row", ctypes.c_double),
                ("sigma_ref_col", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class H2Profile(ctypes.Structure):
    _fields_ = [("calls", ctypes.c_int64)] + [(name, ctypes.c_double) for name in (
        "ms_permute", "ms_upsweep", "ms_coupling", "ms_downsweep", "ms_dense", "ms_leaf_out", "ms_total")]

    def as_dict(self):
        return {name: (int if name == "calls" else float)(getattr(self, name)) for name, _ in self._fields_}


class H2BatchItem(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("ldx", ctypes.c_int64), ("Y", ctypes.c_void_p), ("ldy", ctypes.c_int64),
                ("nv", ctypes.c_int64), ("alpha", ctypes.c_double), ("beta", ctypes.c_double)]


class H2ServerStats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "submitted", "completed", "calls", "vectors", "max_inflight_calls", "slots", "budget_bytes",
        "hbm_free_at_create")] + [("alg_bytes", ctypes.c_double), ("alg_flops", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class H2Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libh2gemv error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libh2gemv.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() -- there is no fallback")
    lib = ctypes.CDLL(path)
    vp, i64, ci, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.h2_load.argtypes = [ctypes.c_char_p, ci, ctypes.POINTER(vp)]
    lib.h2_load.restype = ci
    lib.h2_load_mem.argtypes = [vp, ctypes.c_size_t, ci, ctypes.POINTER(vp)]
    lib.h2_load_mem.restype = ci
    lib.h2_validate.argtypes = [vp, ctypes.c_size_t]
    lib.h2_validate.restype = ci
    lib.h2_gemv.argtypes = [vp, ctypes.c_char, dbl, vp, i64, i64, dbl, vp, i64, vp]
    lib.h2_gemv.restype = ci
    lib.h2_gemv_ex.argtypes = [vp, ctypes.c_char, dbl, vp, i64, i64, dbl, vp, i64, ci, vp]
    lib.h2_gemv_ex.restype = ci
    lib.h2_gemv_noalloc.argtypes = [vp, ctypes.c_char, dbl, vp, i64, i64, dbl, vp, i64, vp]
    lib.h2_gemv_noalloc.restype = ci
    lib.h2_graph.argtypes = [vp, ci]
    lib.h2_graph.restype = ci
    lib.h2_prepare.argtypes = [vp, ci]
    lib.h2_prepare.restype = ci
    lib.h2_reserve.argtypes = [vp, i64]
    lib.h2_reserve.restype = ci
    lib.h2_tune.argtypes = [vp, i64, ci, vp]
    lib.h2_tune.restype = ci
    lib.h2_compress.argtypes = [vp, dbl, ctypes.POINTER(vp), ctypes.POINTER(H2CompressInfo), vp]
    lib.h2_compress.restype = ci
    lib.h2_export.argtypes = [vp, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
    lib.h2_export.restype = ci
    lib.h2_ranks.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), i64]
    lib.h2_ranks.restype = ci
    lib.h2_plan_info.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
    lib.h2_plan_info.restype = ci
    lib.h2_tune_set.argtypes = [vp, ci, ci, i64, ci, ci]
    lib.h2_tune_set.restype = ci
    lib.h2_set_dense_grid.argtypes = [vp, i64]
    lib.h2_set_dense_grid.restype = ci
    lib.h2_set_sweeps.argtypes = [vp, ci, ci]
    lib.h2_set_sweeps.restype = ci
    lib.h2_set_fragment_order.argtypes = [vp, ci, ci]
    lib.h2_set_fragment_order.restype = ci
    lib.h2_set_schedule.argtypes = [vp, ci, ci]
    lib.h2_set_schedule.restype = ci
    lib.h2_stats.argtypes = [vp, ctypes.POINTER(H2Stats)]
    lib.h2_stats.restype = ci
    lib.h2_level_stats.argtypes = [vp, i64, ctypes.POINTER(H2LevelStats)]
    lib.h2_level_stats.restype = ci
    lib.h2_n.argtypes = [vp]
    lib.h2_n.restype = i64
    lib.h2_profile.argtypes = [vp, ci]
    lib.h2_profile.restype = ci
    lib.h2_profile_read.argtypes = [vp, ctypes.POINTER(H2Profile)]
    lib.h2_profile_read.restype = ci
    lib.h2_batch_load.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_size_t), i64, i64, ci,
                                  ctypes.POINTER(vp)]
    lib.h2_batch_load.restype = ci
    lib.h2_batch_load_ex.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_size_t), i64, ctypes.POINTER(i64),
                                     ci, ctypes.POINTER(vp)]
    lib.h2_batch_load_ex.restype = ci
    lib.h2_batch_gemv.argtypes = [vp, ctypes.POINTER(H2BatchItem), vp]
    lib.h2_batch_gemv.restype = ci
    lib.h2_batch_tune.argtypes = [vp, ctypes.POINTER(H2BatchItem), vp]
    lib.h2_batch_tune.restype = ci
    lib.h2_batch_graph.argtypes = [vp, ci]
    lib.h2_batch_graph.restype = ci
    lib.h2_batch_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(dbl),
                                  ctypes.POINTER(i64)]
    lib.h2_batch_info.restype = ci
    lib.h2_batch_plan_info.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
    lib.h2_batch_plan_info.restype = ci
    lib.h2_batch_free.argtypes = [vp]
    lib.h2_batch_free.restype = ci
    lib.h2_server_create.argtypes = [ctypes.POINTER(vp), i64, i64, i64, i64, ctypes.POINTER(vp)]
    lib.h2_server_create.restype = ci
    lib.h2_server_submit.argtypes = [vp, i64, ci, i64, vp, vp, vp, ctypes.POINTER(i64)]
    lib.h2_server_submit.restype = ci
    lib.h2_server_wait.argtypes = [vp, i64, ctypes.POINTER(dbl)]
    lib.h2_server_wait.restype = ci
    lib.h2_server_stats.argtypes = [vp, ctypes.POINTER(H2ServerStats)]
    lib.h2_server_stats.restype = ci
    lib.h2_server_free.argtypes = [vp]
    lib.h2_server_free.restype = ci
    lib.h2_free.argtypes = [vp]
    lib.h2_free.restype = ci
    lib.h2_last_error.argtypes = []
    lib.h2_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc):
    if rc != H2_OK:
        raise H2Error(rc, load_library().h2_last_error().decode(errors="replace"))


def validate(buf) -> int:
    """Host-only validation of a serialized representation; returns the code."""
    b = np.ascontiguousarray(np.asarray(buf).view(np.uint8).ravel())
    return int(load_library().h2_validate(b.ctypes.data, b.size))


class H2Operator:
    """One H^2 operator resident on a GPU.

    ``src`` is a path to a serialized representation or a uint8 buffer
    holding one.  ``gemv`` computes Y <- alpha op(A) X + beta Y for device
    tensors X, Y of shape (n, nv) in column-major layout (stride (1, ld)).
    """

    def __init__(self, src, device: int = 0):
        lib = load_library()
        h = ctypes.c_void_p()
        if isinstance(src, ctypes.c_void_p):  # an existing handle (owned from now on)
            h = src
        elif isinstance(src, (str, os.PathLike)):
            _check(lib.h2_load(os.fsencode(src), device, ctypes.byref(h)))
        else:
            b = np.ascontiguousarray(np.asarray(src).view(np.uint8).ravel())
            _check(lib.h2_load_mem(b.ctypes.data, b.size, device, ctypes.byref(h)))
        self._h = h
        self.device = device
        self.n = int(lib.h2_n(h))

    def close(self):
        if getattr(self, "_h", None):
            load_library().h2_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def compress(self, tau: float, stream: int = 0):
        """Algebraic recompression to threshold tau: (new operator, info)."""
        h = ctypes.c_void_p()
        info = H2CompressInfo()
        _check(load_library().h2_compress(self._h, float(tau), ctypes.byref(h), ctypes.byref(info),
                                          stream or None))
        return H2Operator(h, self.device), info.as_dict()

    def export(self) -> np.ndarray:
        """The serialized representation (uint8 array, no points)."""
        lib = load_library()
        need = ctypes.c_size_t()
        _check(lib.h2_export(self._h, None, 0, ctypes.byref(need)))
        buf = np.zeros(need.value // 8 + 1, dtype=np.uint64).view(np.uint8)[:need.value]
        _check(lib.h2_export(self._h, buf.ctypes.data, buf.size, ctypes.byref(need)))
        return buf

    def tune_set(self, precision: str = "fp64", kc: int = 64, grid: int = 0, xcd: bool = False,
                 tree_order: int = 0):
        """Fixed multi-vector launch parameters for every launch (see h2_tune_set)."""
        _check(load_library().h2_tune_set(self._h, PRECISIONS[precision], kc, grid, 1 if xcd else 0,
                                          int(tree_order)))

    def set_dense_grid(self, workgroups: int = -1):
        """Workgroups of the multi-vector dense launches (see h2_set_dense_grid)."""
        _check(load_library().h2_set_dense_grid(self._h, int(workgroups)))

    def set_schedule(self, precision: str = "fp64", schedule: int = 0):
        """Where the multi-vector dense and coupling rows run, 0-3 (see h2_set_schedule)."""
        _check(load_library().h2_set_schedule(self._h, PRECISIONS[precision], int(schedule)))

    def set_sweeps(self, precision: str = "fp64", fused: bool = True):
        """Fused subtree sweeps or one launch per level (see h2_set_sweeps)."""
        _check(load_library().h2_set_sweeps(self._h, PRECISIONS[precision], 1 if fused else 0))

    def set_fragment_order(self, precision: str = "fp64", enable: bool = True):
        """Wave-row launches read the fragment-ordered matrix copy (see h2_set_fragment_order)."""
        _check(load_library().h2_set_fragment_order(self._h, PRECISIONS[precision], 1 if enable else 0))

    def plan_info(self) -> str:
        """Text description of the launch plan and its tuned parameters."""
        lib = load_library()
        need = ctypes.c_size_t()
        _check(lib.h2_plan_info(self._h, None, 0, ctypes.byref(need)))
        buf = ctypes.create_string_buffer(need.value)
        _check(lib.h2_plan_info(self._h, buf, need.value, ctypes.byref(need)))
        return buf.value.decode()

    def ranks(self):
        """Row and column ranks per level."""
        depth = self.stats()["depth"]
        kr = (ctypes.c_int64 * (depth + 1))()
        kc = (ctypes.c_int64 * (depth + 1))()
        _check(load_library().h2_ranks(self._h, kr, kc, depth + 1))
        return np.array(kr[:], dtype=np.int64), np.array(kc[:], dtype=np.int64)

    def stats(self) -> dict:
        st = H2Stats()
        _check(load_library().h2_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def level_stats(self) -> list:
        """Per-level structure, root first (see h2_level_stats)."""
        out = []
        for level in range(self.stats()["depth"] + 1):
            ls = H2LevelStats()
            _check(load_library().h2_level_stats(self._h, level, ctypes.byref(ls)))
            out.append(ls.as_dict())
        return out

    def reserve(self, nv_max: int):
        _check(load_library().h2_reserve(self._h, nv_max))

    def profile(self, enable: bool = True):
        _check(load_library().h2_profile(self._h, 1 if enable else 0))

    def profile_read(self) -> dict:
        p = H2Profile()
        _check(load_library().h2_profile_read(self._h, ctypes.byref(p)))
        return p.as_dict()

    def graph(self, enable: bool = True):
        """Replay repeated products on the same buffers from captured HIP graphs (see h2_graph)."""
        _check(load_library().h2_graph(self._h, 1 if enable else 0))

    def prepare(self, precision: str):
        _check(load_library().h2_prepare(self._h, PRECISIONS[precision]))

    def tune(self, nv: int, precision: str = "fp64", stream: int = 0):
        """Autotune the multi-vector path for nv vectors (synchronous)."""
        _check(load_library().h2_tune(self._h, nv, PRECISIONS[precision], stream or None))

    def gemv_raw(self, op: str, alpha: float, x_ptr: int, ldx: int, nv: int, beta: float, y_ptr: int,
                 ldy: int, stream: int = 0, precision: str = "fp64"):
        """Direct C-ABI call with device pointers (integers)."""
        lib = load_library()
        if precision == "fp64":
            _check(lib.h2_gemv(self._h, op.encode(), float(alpha), x_ptr or None, ldx, nv, float(beta),
                               y_ptr or None, ldy, stream or None))
        else:
            _check(lib.h2_gemv_ex(self._h, op.encode(), float(alpha), x_ptr or None, ldx, nv, float(beta),
                                  y_ptr or None, ldy, PRECISIONS[precision], stream or None))

    def gemv(self, X, op: str = "N", alpha: float = 1.0, beta: float = 0.0, Y=None, stream=None,
             precision: str = "fp64"):
        """Y <- alpha op(A) X + beta Y.  X, Y: torch tensors (device or host;
        host tensors are copied to the operator's device).  Returns Y."""
        import torch
        dev = torch.device("cuda", self.device)

        def colmajor(t):
            t = t.to(device=dev, dtype=torch.float64)
            if t.dim() == 1:
                t = t.reshape(-1, 1)
            if t.shape[0] != self.n:
                raise ValueError(f"expected {self.n} rows, got {t.shape[0]}")
            if t.stride(0) != 1 or (t.shape[1] > 1 and t.stride(1) < self.n):
                t = t.t().contiguous().t()
            return t

        s = stream if stream is not None else torch.cuda.current_stream(dev)
        with torch.cuda.stream(s):
            X = colmajor(X)
            nv = X.shape[1]
            Y_in = Y
            if Y is None:
                Y = torch.empty((nv, self.n), dtype=torch.float64, device=dev).t()
                beta = 0.0
            else:
                Y = colmajor(Y)
            ldx = X.stride(1) if nv > 1 else self.n
            ldy = Y.stride(1) if nv > 1 else self.n
            self.gemv_raw(op, alpha, X.data_ptr(), ldx, nv, beta, Y.data_ptr(), ldy, s.cuda_stream, precision)
            if Y_in is not None and Y.data_ptr() != Y_in.data_ptr():
                # Y was converted to a column-major FP64 device copy: write
                # the result back into the caller's tensor (in place)
                Y_in.copy_(Y.reshape(Y_in.shape))
                return Y_in
        return Y


class H2Batch:
    """Several operators applied together by merged launches (op 'N', FP64).

    ``bufs``: list of uint8 buffers holding serialized representations;
    ``nv_max``: the largest vector count of any call, one for all operators
    or one per operator.  ``gemv(Xs, Ys, nvs, alphas, betas)`` takes
    per-operator device tensors (column-major n_i x nv_i) and computes
    Y_i <- alpha_i A_i X_i + beta_i Y_i.
    """

    def __init__(self, bufs, nv_max, device: int = 0):
        lib = load_library()
        self._keep = [np.ascontiguousarray(np.asarray(b).view(np.uint8).ravel()) for b in bufs]
        ptrs = (ctypes.c_void_p * len(bufs))(*[b.ctypes.data for b in self._keep])
        lens = (ctypes.c_size_t * len(bufs))(*[b.size for b in self._keep])
        nvm = [int(nv_max)] * len(bufs) if np.isscalar(nv_max) else [int(v) for v in nv_max]
        if len(nvm) != len(bufs):
            raise ValueError("one nv_max per operator")
        h = ctypes.c_void_p()
        _check(lib.h2_batch_load_ex(ptrs, lens, len(bufs), (ctypes.c_int64 * len(nvm))(*nvm), device,
                                    ctypes.byref(h)))
        self._keep = None  # only read during the load
        self._h = h
        self.count = len(bufs)
        self.nv_max = nvm
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            load_library().h2_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        c, n, l = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        f = ctypes.c_double()
        _check(load_library().h2_batch_info(self._h, ctypes.byref(c), ctypes.byref(n), ctypes.byref(f),
                                            ctypes.byref(l)))
        return {"count": c.value, "total_n": n.value, "flops_per_vector": f.value, "launches": l.value}

    def plan_info(self) -> str:
        """Text description of the merged launches and their tuned parameters."""
        lib = load_library()
        need = ctypes.c_size_t()
        _check(lib.h2_batch_plan_info(self._h, None, 0, ctypes.byref(need)))
        buf = ctypes.create_string_buffer(need.value)
        _check(lib.h2_batch_plan_info(self._h, buf, need.value, ctypes.byref(need)))
        return buf.value.decode()

    @staticmethod
    def _items(Xs, Ys, alphas, betas):
        items = (H2BatchItem * len(Xs))()
        for i, (X, Y) in enumerate(zip(Xs, Ys)):
            nv = 0 if Y is None else (Y.shape[1] if Y.dim() > 1 else 1)
            n = 0 if Y is None else Y.shape[0]
            items[i] = H2BatchItem(None if X is None else X.data_ptr(), (X.stride(1) if X is not None and nv > 1 else n),
                                   None if Y is None else Y.data_ptr(), (Y.stride(1) if Y is not None and nv > 1 else n),
                                   nv, float(alphas[i]), float(betas[i]))
        return items

    def gemv(self, Xs, Ys, alphas=None, betas=None, stream=None):
        import torch
        alphas = alphas if alphas is not None else [1.0] * len(Xs)
        betas = betas if betas is not None else [0.0] * len(Xs)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        _check(load_library().h2_batch_gemv(self._h, self._items(Xs, Ys, alphas, betas), s.cuda_stream))

    def tune(self, Xs, Ys, alphas=None, betas=None, stream=None):
        import torch
        alphas = alphas if alphas is not None else [1.0] * len(Xs)
        betas = betas if betas is not None else [0.0] * len(Xs)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        _check(load_library().h2_batch_tune(self._h, self._items(Xs, Ys, alphas, betas), s.cuda_stream))

    def graph(self, enable: bool = True):
        _check(load_library().h2_batch_graph(self._h, 1 if enable else 0))


class H2Server:
    """Serving loop over resident operators (continuous batching in C++).

    ``submit(op, X, precision)`` queues Y = A_op X for a device tensor X
    (n x nv; any layout: a column-major copy is made on the current stream)
    and returns a request id.  The server reads X after the work queued on
    the current stream so far, so X may still be in production.  The output
    tensor is allocated here and returned by ``wait(id)`` together with the
    request's latency in ms.  ``budget_bytes`` <= 0 takes a quarter of the
    free HBM."""

    def __init__(self, ops, slots: int = 4, budget_bytes: int = 1 << 30, max_fuse_nv: int = 64):
        lib = load_library()
        self._ops = list(ops)
        hs = (ctypes.c_void_p * len(self._ops))(*[o._h.value for o in self._ops])
        h = ctypes.c_void_p()
        _check(lib.h2_server_create(hs, len(self._ops), slots, budget_bytes, max_fuse_nv, ctypes.byref(h)))
        self._h = h
        self._live = {}

    def submit(self, op: int, X, precision: str = "fp64") -> int:
        import torch
        n = self._ops[op].n
        X = X.reshape(n, -1) if X.dim() == 1 else X
        X = X.to(dtype=torch.float64)
        if X.stride(0) != 1 or (X.shape[1] > 1 and X.stride(1) != n):
            X = X.t().contiguous().t()
        nv = X.shape[1]
        Y = torch.empty((nv, n), dtype=torch.float64, device=X.device).t()
        rid = ctypes.c_int64()
        stream = torch.cuda.current_stream(X.device).cuda_stream
        _check(load_library().h2_server_submit(self._h, op, PRECISIONS[precision], nv, X.data_ptr(), Y.data_ptr(),
                                               stream or None, ctypes.byref(rid)))
        self._live[rid.value] = (X, Y)
        return rid.value

    def wait(self, rid: int):
        lat = ctypes.c_double()
        _check(load_library().h2_server_wait(self._h, rid, ctypes.byref(lat)))
        X, Y = self._live.pop(rid)
        return Y, lat.value

    def stats(self) -> dict:
        st = H2ServerStats()
        _check(load_library().h2_server_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            load_library().h2_server_free(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


__all__ = ["H2CompressInfo", "H2Operator", "H2Batch", "H2Server", "H2Error", "load_library", "validate", "EXPORTS"]
