"""Tiny random H^2 representations for exactness and structure tests.

A random cluster tree of uniform depth (any arity, possibly empty leaves), a
random block partition from a random dual-tree traversal, separate row and
column bases with their own ranks per level, and entries drawn either as small
integers (so every partial sum is exact in FP64) or as standard normals.
"""
from __future__ import annotations

import numpy as np

from . import fmt


def random_rep(seed: int, q: int = 2, max_children: int = 3, max_leaf: int = 4,
               max_rank: int = 3, p_adm: float = 0.4, integer: bool = True,
               separate: bool = True, int_range: int = 2, allow_empty: bool = True,
               ranks=None) -> np.ndarray:
    rng = np.random.default_rng(seed)
    # ---- tree: level-major, children of a parent contiguous and in parent order
    levels = [[0]]
    parent = [-1]
    sizes_children = []
    for l in range(q):
        nxt = []
        for t in levels[l]:
            nc = int(rng.integers(1, max_children + 1))
            for _ in range(nc):
                nxt.append(len(parent))
                parent.append(t)
        levels.append(nxt)
    nnodes = len(parent)
    leaves = levels[q]
    lo_leaf = 0 if allow_empty else 1
    msz = rng.integers(lo_leaf, max_leaf + 1, size=len(leaves))
    if msz.sum() == 0:
        msz[0] = 1
    n = int(msz.sum())
    lo = np.zeros(nnodes, np.int64); hi = np.zeros(nnodes, np.int64)
    pos = 0
    for j, t in enumerate(leaves):
        lo[t] = pos; pos += int(msz[j]); hi[t] = pos
    for l in range(q - 1, -1, -1):
        for t in levels[l]:
            ch = [c for c in levels[l + 1] if parent[c] == t]
            lo[t] = lo[ch[0]]; hi[t] = hi[ch[-1]]
    level_ptr = np.cumsum([0] + [len(x) for x in levels]).astype(np.int64)
    children = [[] for _ in range(nnodes)]
    for c in range(1, nnodes):
        children[parent[c]].append(c)

    if ranks is None:
        krow = rng.integers(1, max_rank + 1, size=q + 1)
        kcol = rng.integers(1, max_rank + 1, size=q + 1) if separate else krow.copy()
    else:
        krow, kcol = np.asarray(ranks[0]), np.asarray(ranks[1] if separate else ranks[0])

    def draw(shape):
        if integer:
            return rng.integers(-int_range, int_range + 1, size=shape).astype(np.float64)
        return rng.standard_normal(shape)

    # ---- block partition by random dual traversal
    adm = [[] for _ in range(q + 1)]
    dense = []
    cur = [(0, 0)]
    for l in range(q + 1):
        nxt = []
        for (t, s) in cur:
            if rng.random() < p_adm:
                adm[l].append((t, s))
            elif l == q:
                dense.append((t, s))
            else:
                for a in children[t]:
                    for b in children[s]:
                        nxt.append((a, b))
        cur = nxt
    s_rowptr, s_col = [], []
    for l in range(q + 1):
        first = int(level_ptr[l]); nl = int(level_ptr[l + 1] - first)
        blocks = sorted(adm[l])
        rp = np.zeros(nl + 1, np.int64)
        for (t, s) in blocks:
            rp[t - first + 1] += 1
        s_rowptr.append(np.cumsum(rp))
        s_col.append(np.array([s - first for (t, s) in blocks], np.int64))
        adm[l] = blocks
    dense.sort()
    leaf0 = int(level_ptr[q]); nleaves = len(leaves)
    drp = np.zeros(nleaves + 1, np.int64)
    for (t, s) in dense:
        drp[t - leaf0 + 1] += 1
    d_rowptr = np.cumsum(drp)
    d_col = np.array([s - leaf0 for (t, s) in dense], np.int64)

    U = draw(n * int(krow[q]))
    E = np.concatenate([draw(int(krow[l]) * int(krow[l - 1]))
                        for l in range(1, q + 1) for _ in levels[l]]) if q else np.zeros(0)
    V = draw(n * int(kcol[q])) if separate else None
    F = (np.concatenate([draw(int(kcol[l]) * int(kcol[l - 1]))
                         for l in range(1, q + 1) for _ in levels[l]]) if q else np.zeros(0)) if separate else None
    S = np.concatenate([draw(int(krow[l]) * int(kcol[l])) for l in range(q + 1) for _ in adm[l]] or [np.zeros(0)])
    D = np.concatenate([draw(int(hi[t] - lo[t]) * int(hi[s] - lo[s])) for (t, s) in dense] or [np.zeros(0)])
    perm = rng.permutation(n).astype(np.int64)
    rep = dict(n=n, q=q, level_ptr=level_ptr, krow=krow, kcol=kcol, perm=perm, lo=lo, hi=hi,
               parent=np.array(parent, np.int64), s_rowptr=s_rowptr, s_col=s_col,
               d_rowptr=d_rowptr, d_col=d_col, U=U, E=E, S=S, D=D)
    if separate:
        rep["V"] = V; rep["F"] = F
    return fmt.write(rep)
