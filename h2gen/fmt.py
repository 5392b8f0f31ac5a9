"""Serialized H^2 representation (``.h2``, version 1): Python writer and parser.

This module belongs to the seeded input generator.  It holds no part of the
matrix-vector arithmetic; it only lays out and reads back the arrays that
describe one H^2 matrix  A = A_de + <U, S, V^T>  (Section 2.1 of the paper:
nested row/column bases with explicit leaf bases and interlevel transfer
matrices, a matrix tree of coupling blocks, and a block-sparse set of dense
leaf blocks).

Layout (little-endian; every array is 8-byte elements; every section starts on
a 64-byte boundary; matrices are column-major):

  header (128 bytes)
     0  char[8]  magic  b"H2MATV01"
     8  u32      version = 1
    12  u32      flags: bit0 = separate column basis (V, F stored);
                        bit1 = points stored
    16  i64      n        matrix order (rows = columns = points)
    24  i64      q        leaf level (root is level 0; every leaf is on level q)
    32  i64      nnodes   nodes of the cluster tree, level-major numbering
    40  i64      dim      point dimension (0 when no points are stored)
    48  i64      kernel_id      (metadata)
    56  f64      kernel_param   (metadata)
    64  f64      eta            (metadata)
    72  i64      cheb_p         (metadata)
    80  i64      leaf_size      (metadata)
    88  i64      ndense   number of dense leaf blocks
    96  i64      total_bytes
   104  zero padding to 128

  sections, in this order
     level_ptr  i64[q+2]   nodes of level l are [level_ptr[l], level_ptr[l+1])
     krow       i64[q+1]   row-basis rank per level
     kcol       i64[q+1]   column-basis rank per level
     nadm       i64[q+1]   coupling blocks per level
     perm       i64[n]     tree position -> original index
     lo, hi     i64[nnodes] each: tree-ordered index range of each node
     parent     i64[nnodes] (root: -1)
     s_rowptr   i64[nnodes+q+1]  per level l, nodes_l+1 entries (CSR row pointer)
     s_col      i64[sum nadm]    level-local column node of each coupling block
     d_rowptr   i64[nleaves+1]   CSR over leaf rows
     d_col      i64[ndense]      leaf-local column index of each dense block
     U          f64[n*krow[q]]   leaf t: m_t x krow[q] at offset lo_t*krow[q]
     E          f64[...]         node c on level l>=1: krow[l] x krow[l-1], node order
     V, F       as U, E with kcol (empty unless flags bit0)
     S          f64[...]         blocks krow[l] x kcol[l] in CSR order, level by level
     D          f64[...]         blocks m_t x m_s in CSR order
     points     f64[n*dim]       original order, point-major (empty unless bit1)
"""
from __future__ import annotations

import numpy as np

MAGIC = b"H2MATV01"
VERSION = 1
HEADER_BYTES = 128
ALIGN = 64
FLAG_SEPARATE_V = 1
FLAG_POINTS = 2

SECTION_NAMES = (
    "level_ptr", "krow", "kcol", "nadm", "perm", "lo", "hi", "parent",
    "s_rowptr", "s_col", "d_rowptr", "d_col",
    "U", "E", "V", "F", "S", "D", "points",
)
_INT_SECTIONS = set(SECTION_NAMES[:12])


def _align(x: int) -> int:
    return (x + ALIGN - 1) // ALIGN * ALIGN


def section_sizes(n, q, nnodes, flags, dim, level_ptr, krow, kcol, nadm,
                  lo, hi, d_rowptr, d_col):
    """Element count of every section, derived from the structural arrays."""
    nodes = [int(level_ptr[l + 1] - level_ptr[l]) for l in range(q + 1)]
    nleaves = nodes[q]
    sep = bool(flags & FLAG_SEPARATE_V)
    e_sz = sum(nodes[l] * int(krow[l]) * int(krow[l - 1]) for l in range(1, q + 1))
    f_sz = sum(nodes[l] * int(kcol[l]) * int(kcol[l - 1]) for l in range(1, q + 1))
    s_sz = sum(int(nadm[l]) * int(krow[l]) * int(kcol[l]) for l in range(q + 1))
    leaf0 = int(level_ptr[q])
    d_sz = 0
    if d_rowptr is not None:
        m = np.asarray(hi[leaf0:], dtype=np.int64) - np.asarray(lo[leaf0:], dtype=np.int64)
        for t in range(nleaves):
            for b in range(int(d_rowptr[t]), int(d_rowptr[t + 1])):
                d_sz += int(m[t]) * int(m[int(d_col[b])])
    return {
        "level_ptr": q + 2, "krow": q + 1, "kcol": q + 1, "nadm": q + 1,
        "perm": n, "lo": nnodes, "hi": nnodes, "parent": nnodes,
        "s_rowptr": nnodes + q + 1, "s_col": int(sum(int(x) for x in nadm)),
        "d_rowptr": nleaves + 1, "d_col": len(d_col),
        "U": n * int(krow[q]), "E": e_sz,
        "V": n * int(kcol[q]) if sep else 0, "F": f_sz if sep else 0,
        "S": s_sz, "D": d_sz,
        "points": n * dim if flags & FLAG_POINTS else 0,
    }


def write(rep: dict) -> np.ndarray:
    """Serialize a representation given as a dict of arrays; returns uint8 array.

    Required keys: n, q, level_ptr, krow, kcol, perm, lo, hi, parent,
    s_rowptr (list over levels), s_col (list over levels), d_rowptr, d_col,
    U, E, S, D.  Optional: V, F (separate column basis), points, and metadata
    kernel_id, kernel_param, eta, cheb_p, leaf_size.
    """
    n = int(rep["n"]); q = int(rep["q"])
    level_ptr = np.asarray(rep["level_ptr"], dtype=np.int64)
    nnodes = int(level_ptr[q + 1])
    krow = np.asarray(rep["krow"], dtype=np.int64)
    kcol = np.asarray(rep["kcol"], dtype=np.int64)
    s_rowptr = [np.asarray(r, dtype=np.int64) for r in rep["s_rowptr"]]
    s_col = [np.asarray(c, dtype=np.int64) for c in rep["s_col"]]
    nadm = np.array([len(c) for c in s_col], dtype=np.int64)
    d_rowptr = np.asarray(rep["d_rowptr"], dtype=np.int64)
    d_col = np.asarray(rep["d_col"], dtype=np.int64)
    sep = rep.get("V") is not None
    pts = rep.get("points")
    flags = (FLAG_SEPARATE_V if sep else 0) | (FLAG_POINTS if pts is not None else 0)
    dim = int(np.asarray(pts).shape[1]) if pts is not None else 0
    data = {
        "level_ptr": level_ptr, "krow": krow, "kcol": kcol, "nadm": nadm,
        "perm": np.asarray(rep["perm"], dtype=np.int64),
        "lo": np.asarray(rep["lo"], dtype=np.int64),
        "hi": np.asarray(rep["hi"], dtype=np.int64),
        "parent": np.asarray(rep["parent"], dtype=np.int64),
        "s_rowptr": np.concatenate(s_rowptr) if s_rowptr else np.zeros(0, np.int64),
        "s_col": np.concatenate(s_col) if s_col else np.zeros(0, np.int64),
        "d_rowptr": d_rowptr, "d_col": d_col,
        "U": np.asarray(rep["U"], dtype=np.float64).ravel(order="K"),
        "E": np.asarray(rep["E"], dtype=np.float64).ravel(order="K"),
        "V": np.asarray(rep["V"], dtype=np.float64).ravel(order="K") if sep else np.zeros(0),
        "F": np.asarray(rep["F"], dtype=np.float64).ravel(order="K") if sep else np.zeros(0),
        "S": np.asarray(rep["S"], dtype=np.float64).ravel(order="K"),
        "D": np.asarray(rep["D"], dtype=np.float64).ravel(order="K"),
        "points": np.ascontiguousarray(pts, dtype=np.float64).ravel() if pts is not None else np.zeros(0),
    }
    want = section_sizes(n, q, nnodes, flags, dim, level_ptr, krow, kcol, nadm,
                         data["lo"], data["hi"], d_rowptr, d_col)
    for name in SECTION_NAMES:
        if data[name].size != want[name]:
            raise ValueError(f"section {name}: {data[name].size} elements, expected {want[name]}")
    offs = {}
    pos = HEADER_BYTES
    for name in SECTION_NAMES:
        pos = _align(pos)
        offs[name] = pos
        pos += 8 * data[name].size
    total = _align(pos)
    buf = np.zeros(total, dtype=np.uint8)
    hdr = buf[:HEADER_BYTES]
    hdr[:8] = np.frombuffer(MAGIC, dtype=np.uint8)
    hdr[8:16].view(np.uint32)[:] = [VERSION, flags]
    ints = hdr[16:48].view(np.int64)
    ints[:] = [n, q, nnodes, dim]
    hdr[48:56].view(np.int64)[0] = int(rep.get("kernel_id", 0))
    hdr[56:72].view(np.float64)[:] = [float(rep.get("kernel_param", 0.0)), float(rep.get("eta", 0.0))]
    hdr[72:104].view(np.int64)[:] = [int(rep.get("cheb_p", 0)), int(rep.get("leaf_size", 0)),
                                     d_col.size, total]
    for name in SECTION_NAMES:
        arr = data[name]
        if arr.size:
            dt = np.int64 if name in _INT_SECTIONS else np.float64
            buf[offs[name]:offs[name] + 8 * arr.size].view(dt)[:] = arr
    return buf


def parse(buf) -> dict:
    """Zero-copy parse of a serialized representation into numpy views.

    Checks the magic, version, flags and total size only; structural validity
    is the business of the consumers' own readers.
    """
    b = np.frombuffer(buf, dtype=np.uint8) if not isinstance(buf, np.ndarray) else buf.view(np.uint8).ravel()
    if b.size < HEADER_BYTES or bytes(b[:8]) != MAGIC:
        raise ValueError("not an H2 representation (bad magic)")
    version, flags = (int(x) for x in b[8:16].view(np.uint32))
    if version != VERSION:
        raise ValueError(f"unsupported version {version}")
    n, q, nnodes, dim = (int(x) for x in b[16:48].view(np.int64))
    kernel_id = int(b[48:56].view(np.int64)[0])
    kernel_param, eta = (float(x) for x in b[56:72].view(np.float64))
    cheb_p, leaf_size, ndense, total = (int(x) for x in b[72:104].view(np.int64))
    if total != b.size:
        raise ValueError(f"size mismatch: header says {total}, buffer has {b.size}")
    out = dict(n=n, q=q, nnodes=nnodes, dim=dim, flags=flags, kernel_id=kernel_id,
               kernel_param=kernel_param, eta=eta, cheb_p=cheb_p, leaf_size=leaf_size,
               ndense=ndense, total_bytes=total)
    pos = HEADER_BYTES

    def take(count, dt):
        nonlocal pos
        pos = _align(pos)
        a = b[pos:pos + 8 * count].view(dt)
        pos += 8 * count
        return a

    out["level_ptr"] = take(q + 2, np.int64)
    out["krow"] = take(q + 1, np.int64)
    out["kcol"] = take(q + 1, np.int64)
    out["nadm"] = take(q + 1, np.int64)
    out["perm"] = take(n, np.int64)
    out["lo"] = take(nnodes, np.int64)
    out["hi"] = take(nnodes, np.int64)
    out["parent"] = take(nnodes, np.int64)
    out["s_rowptr_flat"] = take(nnodes + q + 1, np.int64)
    out["s_col_flat"] = take(int(out["nadm"].sum()), np.int64)
    lp = out["level_ptr"]
    nleaves = int(lp[q + 1] - lp[q])
    out["d_rowptr"] = take(nleaves + 1, np.int64)
    out["d_col"] = take(ndense, np.int64)
    sizes = section_sizes(n, q, nnodes, flags, dim, lp, out["krow"], out["kcol"], out["nadm"],
                          out["lo"], out["hi"], out["d_rowptr"], out["d_col"])
    for name in ("U", "E", "V", "F", "S", "D", "points"):
        out[name] = take(sizes[name], np.float64)
    # split per-level CSR of S
    rp, cl = [], []
    r0 = 0; c0 = 0
    for l in range(q + 1):
        nl = int(lp[l + 1] - lp[l])
        rp.append(out["s_rowptr_flat"][r0:r0 + nl + 1]); r0 += nl + 1
        na = int(out["nadm"][l])
        cl.append(out["s_col_flat"][c0:c0 + na]); c0 += na
    out["s_rowptr"] = rp
    out["s_col"] = cl
    if not flags & FLAG_SEPARATE_V:
        out["V"] = out["U"]; out["F"] = out["E"]
    if flags & FLAG_POINTS:
        out["points"] = out["points"].reshape(n, dim)
    else:
        out["points"] = None
    return out
