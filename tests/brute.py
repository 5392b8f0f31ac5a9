"""Brute-force dense expansion of a serialized H^2 representation, for tiny
inputs only.  Written in the tests, independently of the oracle, straight from
the definition in Section 2.1 of the paper: the explicit basis of an inner node
is the block-diagonal of its children's bases times the stacked transfers, and
every coupling block (t,s) of level l contributes Uhat_t S_ts Vhat_s^T to the
block of rows t and columns s; dense blocks are added as stored.
"""
import numpy as np

from h2gen import fmt


def explicit_bases(r, which):
    """Dict node -> explicit basis (|node| x k_level), by recursion up the tree."""
    q = r["q"]; lp = r["level_ptr"]; lo = r["lo"]; hi = r["hi"]; par = r["parent"]
    B = r["U"] if which == "U" else r["V"]
    T = r["E"] if which == "U" else r["F"]
    k = r["krow"] if which == "U" else r["kcol"]
    basis = {}
    kq = int(k[q])
    for t in range(int(lp[q]), int(lp[q + 1])):
        m = int(hi[t] - lo[t])
        basis[t] = B[int(lo[t]) * kq: int(lo[t]) * kq + m * kq].reshape(kq, m).T.copy() if m else np.zeros((0, kq))
    # transfer of node c (level l >= 1): k[l] x k[l-1] column-major, in node order
    toff = {}
    pos = 0
    for l in range(1, q + 1):
        for c in range(int(lp[l]), int(lp[l + 1])):
            toff[c] = pos
            pos += int(k[l]) * int(k[l - 1])
    for l in range(q, 0, -1):
        for p in range(int(lp[l - 1]), int(lp[l])):
            kids = [c for c in range(int(lp[l]), int(lp[l + 1])) if par[c] == p]
            rows = []
            for c in kids:
                Tc = T[toff[c]: toff[c] + int(k[l]) * int(k[l - 1])].reshape(int(k[l - 1]), int(k[l])).T
                rows.append(basis[c] @ Tc)
            basis[p] = np.vstack(rows) if rows else np.zeros((0, int(k[l - 1])))
    return basis


def dense_tree_order(buf, include_dense=True):
    """The matrix in tree order (with include_dense=False: its low-rank part,
    the sum of the coupling blocks' contributions, only)."""
    r = fmt.parse(buf)
    n, q = r["n"], r["q"]
    lp, lo, hi = r["level_ptr"], r["lo"], r["hi"]
    Uh = explicit_bases(r, "U")
    Vh = explicit_bases(r, "V")
    A = np.zeros((n, n))
    soff = 0
    for l in range(q + 1):
        kr, kc = int(r["krow"][l]), int(r["kcol"][l])
        rp, cl = r["s_rowptr"][l], r["s_col"][l]
        for ti in range(int(lp[l + 1] - lp[l])):
            t = int(lp[l]) + ti
            for b in range(int(rp[ti]), int(rp[ti + 1])):
                s = int(lp[l]) + int(cl[b])
                S = r["S"][soff: soff + kr * kc].reshape(kc, kr).T
                soff += kr * kc
                A[lo[t]:hi[t], lo[s]:hi[s]] += Uh[t] @ S @ Vh[s].T
    doff = 0
    leaf0 = int(lp[q])
    for ti in range(int(lp[q + 1] - lp[q]) if include_dense else 0):
        t = leaf0 + ti
        for b in range(int(r["d_rowptr"][ti]), int(r["d_rowptr"][ti + 1])):
            s = leaf0 + int(r["d_col"][b])
            mt, ms = int(hi[t] - lo[t]), int(hi[s] - lo[s])
            A[lo[t]:hi[t], lo[s]:hi[s]] += r["D"][doff: doff + mt * ms].reshape(ms, mt).T
            doff += mt * ms
    return A, r


def dense_original_order(buf):
    """The matrix in original point order: A[perm[i], perm[j]] = Atree[i, j]."""
    At, r = dense_tree_order(buf)
    perm = np.asarray(r["perm"])
    A = np.zeros_like(At)
    A[np.ix_(perm, perm)] = At
    return A


def coupling_blocks(r):
    """(level, row node, column node) of every coupling block."""
    lp = r["level_ptr"]
    out = []
    for l in range(r["q"] + 1):
        rp, cl = r["s_rowptr"][l], r["s_col"][l]
        for ti in range(int(lp[l + 1] - lp[l])):
            for b in range(int(rp[ti]), int(rp[ti + 1])):
                out.append((l, int(lp[l]) + ti, int(lp[l]) + int(cl[b])))
    return out


def block_row(Alr, r, i, rows=True, cols=False):
    """The part of the low-rank matrix Alr (tree order) that node i's basis
    must represent: with rows, for every coupling block (a, s) whose row node
    a is i or an ancestor of i, the rows of i and the columns of s; with cols,
    transposed, for every block (s, a) whose column node a is i or an
    ancestor, the rows of s and the columns of i."""
    lo, hi, par = r["lo"], r["hi"], r["parent"]
    anc = {i}
    c = i
    while par[c] >= 0:
        c = int(par[c])
        anc.add(c)
    parts = []
    for _, t, s in coupling_blocks(r):
        if rows and t in anc:
            parts.append(Alr[lo[i]:hi[i], lo[s]:hi[s]])
        if cols and s in anc:
            parts.append(Alr[lo[t]:hi[t], lo[i]:hi[i]].T)
    m = int(hi[i] - lo[i])
    return np.hstack(parts) if parts else np.zeros((m, 0))
