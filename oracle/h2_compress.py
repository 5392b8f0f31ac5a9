"""Oracle for algebraic recompression of an H^2 matrix (Section 5 of the paper).

TEST INFRASTRUCTURE.  Only the tests, the package's smoke check and the
benchmark's CPU baseline may import this module; the library never does.

Plain NumPy in FP64.  The steps follow the paper's order and notation, one
node at a time, with LAPACK's QR and SVD (through numpy.linalg) as the only
library primitives:

1. Orthogonalization (Sec. 5, last subsection, "orthogonalize the basis"):
   an upsweep of QR factorizations.  Leaf t: U_t = Q_t R_t, the new leaf basis
   is Q_t.  Inner node p: the stack [R_c E_c] over its children is QR-factored;
   its Q, cut into one block per child, gives the new transfers, its R is R_p.
   Coupling blocks become R_t S_ts R_s^T (row factor, column factor).
2. Reweighting downsweep (Sec. 5.1, the equation for B_i^q): from the root
   down, node i stacks R_{i+} E_i^T (its parent's factor times its transfer)
   over S_ij^T for its own coupling blocks, and keeps the R factor of a QR of
   that stack.  With an orthogonal column basis this R has the same Gram
   matrix as the whole block row of the low-rank part that node i's basis must
   represent (own blocks and every ancestor's blocks restricted to i's rows).
3. Truncation upsweep (Sec. 5.2): leaf t takes the SVD of the reweighed basis
   U_t R_t^T and keeps the left singular vectors whose singular values exceed
   the threshold; T_t = U'_t^T U_t.  Inner node p takes the SVD of the stack
   [T_c E_c R_p^T] over its children, keeps the leading left singular vectors
   (cut per child into the new transfers E'_c) and forms
   T_p = sum_c E'_c^T T_c E_c.
4. Projection (Sec. 5.2, last equation): S'_ts = T_t S_ts T_s^T (row and
   column transforms).  Dense blocks are unchanged.

Readings where the paper is silent (each also listed in the design notes):
* threshold: singular value sigma is kept iff sigma > tau * sigma_ref, with
  sigma_ref the largest singular value over the leaves' reweighed bases of
  that basis tree (the 2-norm of the largest low-rank block row);
* the representation keeps one rank per level: the level's new rank is the
  largest count kept by its nodes, and a node that keeps fewer vectors has
  zero columns after them (its projector is unchanged);
* a factorization with fewer rows than columns (a leaf with fewer points than
  the rank, a stack shorter than the rank) is padded with zero columns of Q
  and zero rows of R, keeping the level's rank;
* a shared basis (V = U, F = E) must represent block rows and block columns,
  so its reweighting stack also holds S_ji for the blocks (j, i) in which the
  node is the column (for a symmetric matrix both halves agree).

The module has its own reader and writer of the serialized format (layout
described in the generator's format module); it does not import the library
or the generator.
"""
from __future__ import annotations

import numpy as np

MAGIC = b"H2MATV01"
_HDR = 128
_ALIGN = 64


def _al(x):
    return (x + _ALIGN - 1) // _ALIGN * _ALIGN


# ---------------------------------------------------------------------------
# reader / writer


def read(buf) -> dict:
    """Representation as per-node matrices (copies; buf is not retained)."""
    b = np.asarray(buf).view(np.uint8).ravel()
    if b.size < _HDR or bytes(b[:8]) != MAGIC:
        raise ValueError("bad magic")
    version, flags = (int(x) for x in b[8:16].view(np.uint32))
    if version != 1:
        raise ValueError("bad version")
    n, q, nnodes, dim = (int(x) for x in b[16:48].view(np.int64))
    meta = dict(kernel_id=int(b[48:56].view(np.int64)[0]),
                kernel_param=float(b[56:64].view(np.float64)[0]),
                eta=float(b[64:72].view(np.float64)[0]),
                cheb_p=int(b[72:80].view(np.int64)[0]),
                leaf_size=int(b[80:88].view(np.int64)[0]))
    ndense = int(b[88:96].view(np.int64)[0])
    pos = _HDR

    def take(cnt, dt):
        nonlocal pos
        pos = _al(pos)
        a = b[pos:pos + 8 * cnt].view(dt).copy()
        if a.size != cnt:
            raise ValueError("truncated")
        pos += 8 * cnt
        return a

    lp = take(q + 2, np.int64)
    krow = take(q + 1, np.int64)
    kcol = take(q + 1, np.int64)
    nadm = take(q + 1, np.int64)
    perm = take(n, np.int64)
    lo = take(nnodes, np.int64)
    hi = take(nnodes, np.int64)
    parent = take(nnodes, np.int64)
    srp = take(nnodes + q + 1, np.int64)
    scol = take(int(nadm.sum()), np.int64)
    nleaves = int(lp[q + 1] - lp[q])
    drp = take(nleaves + 1, np.int64)
    dcol = take(ndense, np.int64)
    sep = bool(flags & 1)
    leaf0 = int(lp[q])
    m = hi[leaf0:] - lo[leaf0:]
    dsz = sum(int(m[t]) * int(m[int(dcol[j])]) for t in range(nleaves) for j in range(int(drp[t]), int(drp[t + 1])))

    def level(c):
        return int(np.searchsorted(lp, c, side="right") - 1)

    def bases(k):
        U = take(n * int(k[q]), np.float64)
        leaves = {}
        for t in range(leaf0, int(lp[q + 1])):
            mt = int(hi[t] - lo[t])
            leaves[t] = U[int(lo[t]) * int(k[q]):(int(lo[t]) + mt) * int(k[q])].reshape(int(k[q]), mt).T.copy()
        esz = sum(int(lp[l + 1] - lp[l]) * int(k[l]) * int(k[l - 1]) for l in range(1, q + 1))
        E = take(esz, np.float64)
        tr, off = {}, 0
        for c in range(int(lp[1]) if q >= 1 else nnodes, nnodes):
            l = level(c)
            sz = int(k[l]) * int(k[l - 1])
            tr[c] = E[off:off + sz].reshape(int(k[l - 1]), int(k[l])).T.copy()
            off += sz
        return leaves, tr

    Uleaf, Etr = bases(krow)
    if sep:
        Vleaf, Ftr = bases(kcol)
    else:
        Vleaf, Ftr = None, None
    ssz = sum(int(nadm[l]) * int(krow[l]) * int(kcol[l]) for l in range(q + 1))
    Sflat = take(ssz, np.float64)
    D = take(dsz, np.float64)
    pts = take(n * dim, np.float64) if flags & 2 else None
    # per-level CSR of S and the blocks in CSR order
    s_rowptr, s_col, S = [], [], []
    r0 = c0 = off = 0
    for l in range(q + 1):
        nl = int(lp[l + 1] - lp[l])
        s_rowptr.append(srp[r0:r0 + nl + 1].copy()); r0 += nl + 1
        na = int(nadm[l])
        s_col.append(scol[c0:c0 + na].copy()); c0 += na
        sz = int(krow[l]) * int(kcol[l])
        S.append([Sflat[off + i * sz: off + (i + 1) * sz].reshape(int(kcol[l]), int(krow[l])).T.copy()
                  for i in range(na)])
        off += na * sz
    children = {p: [] for p in range(nnodes)}
    for c in range(1, nnodes):
        children[int(parent[c])].append(c)
    return dict(n=n, q=q, nnodes=nnodes, dim=dim, flags=flags, meta=meta, level_ptr=lp, krow=krow, kcol=kcol,
                perm=perm, lo=lo, hi=hi, parent=parent, s_rowptr=s_rowptr, s_col=s_col, d_rowptr=drp,
                d_col=dcol, U=Uleaf, E=Etr, V=Vleaf, F=Ftr, S=S, D=D, points=pts, children=children,
                shared=not sep)


def write(rep: dict) -> np.ndarray:
    """Serialize a representation in the layout read() takes."""
    n, q, nnodes = rep["n"], rep["q"], rep["nnodes"]
    lp = np.asarray(rep["level_ptr"], np.int64)
    krow = np.asarray(rep["krow"], np.int64)
    kcol = np.asarray(rep["kcol"], np.int64)
    sep = not rep["shared"]
    leaf0 = int(lp[q])

    def basis_arrays(leaves, tr, k):
        U = np.zeros(n * int(k[q]))
        for t in range(leaf0, int(lp[q + 1])):
            B = leaves[t]
            U[int(rep["lo"][t]) * int(k[q]):int(rep["hi"][t]) * int(k[q])] = B.T.ravel()
        parts = [tr[c].T.ravel() for c in range(int(lp[1]) if q >= 1 else nnodes, nnodes)]
        return U, (np.concatenate(parts) if parts else np.zeros(0))

    U, E = basis_arrays(rep["U"], rep["E"], krow)
    if sep:
        V, F = basis_arrays(rep["V"], rep["F"], kcol)
    else:
        V, F = np.zeros(0), np.zeros(0)
    sparts = [blk.T.ravel() for l in range(q + 1) for blk in rep["S"][l]]
    S = np.concatenate(sparts) if sparts else np.zeros(0)
    nadm = np.array([len(c) for c in rep["s_col"]], np.int64)
    pts = rep.get("points")
    flags = (1 if sep else 0) | (2 if pts is not None else 0)
    ints = [lp, krow, kcol, nadm, np.asarray(rep["perm"], np.int64), np.asarray(rep["lo"], np.int64),
            np.asarray(rep["hi"], np.int64), np.asarray(rep["parent"], np.int64),
            np.concatenate([np.asarray(r, np.int64) for r in rep["s_rowptr"]]),
            np.concatenate([np.asarray(c, np.int64) for c in rep["s_col"]]) if nadm.sum() else np.zeros(0, np.int64),
            np.asarray(rep["d_rowptr"], np.int64), np.asarray(rep["d_col"], np.int64)]
    flts = [U, E, V, F, S, np.asarray(rep["D"], np.float64),
            np.asarray(pts, np.float64).ravel() if pts is not None else np.zeros(0)]
    pos = _HDR
    offs = []
    for a in ints + flts:
        pos = _al(pos)
        offs.append(pos)
        pos += 8 * a.size
    total = _al(pos)
    out = np.zeros(total, np.uint8)
    out[:8] = np.frombuffer(MAGIC, np.uint8)
    out[8:16].view(np.uint32)[:] = [1, flags]
    out[16:48].view(np.int64)[:] = [n, q, nnodes, rep["dim"] if pts is not None else 0]
    meta = rep.get("meta", {})
    out[48:56].view(np.int64)[0] = meta.get("kernel_id", 0)
    out[56:72].view(np.float64)[:] = [meta.get("kernel_param", 0.0), meta.get("eta", 0.0)]
    out[72:104].view(np.int64)[:] = [meta.get("cheb_p", 0), meta.get("leaf_size", 0),
                                     len(rep["d_col"]), total]
    for a, o in zip(ints, offs[:len(ints)]):
        out[o:o + 8 * a.size].view(np.int64)[:] = a
    for a, o in zip(flts, offs[len(ints):]):
        out[o:o + 8 * a.size].view(np.float64)[:] = a
    return out


# ---------------------------------------------------------------------------
# the four steps


def _nodes(rep, l):
    lp = rep["level_ptr"]
    return range(int(lp[l]), int(lp[l + 1]))


def _qr_padded(A, k):
    """Reduced QR A = Q R with Q: rows x k and R: k x k (zero-padded when
    A has fewer rows than k columns)."""
    r = A.shape[0]
    if r == 0:
        return np.zeros((0, k)), np.zeros((k, k))
    Q, R = np.linalg.qr(A, mode="reduced")
    if Q.shape[1] < k:
        Q = np.hstack([Q, np.zeros((r, k - Q.shape[1]))])
        R = np.vstack([R, np.zeros((k - R.shape[0], k))])
    return Q, R


def _r_factor(Z, k):
    """R of a reduced QR of the stack Z (min(rows, k) x k; 0 x k if empty)."""
    if Z.shape[0] == 0:
        return np.zeros((0, k))
    return np.linalg.qr(Z, mode="r")


def orthogonalize_tree(rep, leaves, tr, k):
    """QR upsweep of one basis tree: new leaf bases and transfers (same ranks)
    and the factor R of every node (old explicit basis = new one times R)."""
    q = rep["q"]
    R, nleaf, ntr = {}, {}, {}
    for t in _nodes(rep, q):
        nleaf[t], R[t] = _qr_padded(leaves[t], int(k[q]))
    for l in range(q, 0, -1):
        for p in _nodes(rep, l - 1):
            ch = rep["children"][p]
            kl = int(k[l])
            Z = np.vstack([R[c] @ tr[c] for c in ch]) if ch else np.zeros((0, int(k[l - 1])))
            Q, R[p] = _qr_padded(Z, int(k[l - 1]))
            for i, c in enumerate(ch):
                ntr[c] = Q[i * kl:(i + 1) * kl, :]
    return nleaf, ntr, R


def orthogonalize(rep):
    """Step 1: a representation with orthogonal bases and the same matrix."""
    out = dict(rep)
    out["U"], out["E"], Rr = orthogonalize_tree(rep, rep["U"], rep["E"], rep["krow"])
    if rep["shared"]:
        Rc = Rr
    else:
        out["V"], out["F"], Rc = orthogonalize_tree(rep, rep["V"], rep["F"], rep["kcol"])
    out["S"] = [[Rr[t] @ blk @ Rc[s].T for (t, s), blk in zip(_blocks(rep, l), rep["S"][l])]
                for l in range(rep["q"] + 1)]
    return out


def _blocks(rep, l):
    """(row node, column node) of the coupling blocks of level l in CSR order."""
    lp = rep["level_ptr"]
    rp, cl = rep["s_rowptr"][l], rep["s_col"][l]
    out = []
    for ti in range(int(lp[l + 1] - lp[l])):
        for b in range(int(rp[ti]), int(rp[ti + 1])):
            out.append((int(lp[l]) + ti, int(lp[l]) + int(cl[b])))
    return out


def weights(rep, side):
    """Step 2: reweighting factors R_i of every node of the row (side='row')
    or column (side='col') basis tree, root first."""
    q = rep["q"]
    shared = rep["shared"]
    k = rep["krow"] if side == "row" or shared else rep["kcol"]
    tr = rep["E"] if side == "row" or shared else rep["F"]
    W = {}
    for l in range(q + 1):
        own = {i: [] for i in _nodes(rep, l)}
        for (t, s), blk in zip(_blocks(rep, l), rep["S"][l]):
            if side == "row" or shared:
                own[t].append(blk.T)      # block row t: S_ts^T
            if side == "col" or shared:
                own[s].append(blk)        # block column s: S_ts
        for i in _nodes(rep, l):
            parts = []
            if l >= 1:
                Wp = W[int(rep["parent"][i])]
                if Wp.shape[0]:
                    parts.append(Wp @ tr[i].T)
            parts += own[i]
            Z = np.vstack(parts) if parts else np.zeros((0, int(k[l])))
            W[i] = _r_factor(Z, int(k[l]))
    return W


def truncate_tree(rep, leaves, tr, k, W, tau):
    """Step 3 on one (orthogonal) basis tree: new leaf bases, transfers and
    ranks, the transforms T of every node, the reference singular value and
    every node's kept count."""
    q = rep["q"]
    sig = {}
    left = {}
    for t in _nodes(rep, q):
        Ubar = leaves[t] @ W[t].T
        if Ubar.size:
            Wl, s, _ = np.linalg.svd(Ubar, full_matrices=False)
        else:
            Wl, s = np.zeros((Ubar.shape[0], 0)), np.zeros(0)
        left[t], sig[t] = Wl, s
    sref = max((float(s[0]) for s in sig.values() if s.size), default=0.0)
    eps = tau * sref
    count = {t: int(np.sum(sig[t] > eps)) for t in sig}
    knew = np.zeros(q + 1, np.int64)
    knew[q] = max((count[t] for t in _nodes(rep, q)), default=0)
    nleaf, T = {}, {}
    for t in _nodes(rep, q):
        Un = np.zeros((leaves[t].shape[0], int(knew[q])))
        Un[:, :count[t]] = left[t][:, :count[t]]
        nleaf[t] = Un
        T[t] = Un.T @ leaves[t]
    ntr = {}
    for l in range(q, 0, -1):
        svd = {}
        for p in _nodes(rep, l - 1):
            ch = rep["children"][p]
            rows = [T[c] @ tr[c] @ W[p].T for c in ch]
            M = np.vstack(rows) if rows else np.zeros((0, W[p].shape[0]))
            if M.size:
                Wm, s, _ = np.linalg.svd(M, full_matrices=False)
            else:
                Wm, s = np.zeros((M.shape[0], 0)), np.zeros(0)
            svd[p] = (Wm, s)
            sig[p] = s
            count[p] = int(np.sum(s > eps))
        knew[l - 1] = max((count[p] for p in _nodes(rep, l - 1)), default=0)
        kl = int(knew[l])
        for p in _nodes(rep, l - 1):
            ch = rep["children"][p]
            Wm, _ = svd[p]
            Wn = np.zeros((len(ch) * kl, int(knew[l - 1])))
            Wn[:, :count[p]] = Wm[:, :count[p]]
            Tp = np.zeros((int(knew[l - 1]), int(k[l - 1])))
            for i, c in enumerate(ch):
                ntr[c] = Wn[i * kl:(i + 1) * kl, :]
                Tp += ntr[c].T @ T[c] @ tr[c]
            T[p] = Tp
    return nleaf, ntr, knew, T, sref, count, sig


def compress(buf, tau: float):
    """Recompress a serialized representation to threshold tau (Sec. 5).
    Returns (serialized result, info) where info holds the new ranks, the
    reference singular values, and per node the kept count and the singular
    values its truncation saw."""
    rep = orthogonalize(read(buf))
    Wr = weights(rep, "row")
    out = dict(rep)
    out["U"], out["E"], kr, Tr, sr, cr, gr = truncate_tree(rep, rep["U"], rep["E"], rep["krow"], Wr, tau)
    if rep["shared"]:
        kc, Tc, sc, cc, gc = kr, Tr, sr, cr, gr
    else:
        Wc = weights(rep, "col")
        out["V"], out["F"], kc, Tc, sc, cc, gc = truncate_tree(rep, rep["V"], rep["F"], rep["kcol"], Wc, tau)
    out["krow"], out["kcol"] = kr, kc
    out["S"] = [[Tr[t] @ blk @ Tc[s].T for (t, s), blk in zip(_blocks(rep, l), rep["S"][l])]
                for l in range(rep["q"] + 1)]
    info = dict(krow=kr, kcol=kc, sigma_ref_row=sr, sigma_ref_col=sc, count_row=cr, count_col=cc,
                sigma_row=gr, sigma_col=gc)
    return write(out), info


def lowrank_entries(buf) -> int:
    """Stored low-rank entries (U, E, V, F, S) of a serialized representation."""
    r = read(buf)
    tot = sum(b.size for b in r["U"].values()) + sum(b.size for b in r["E"].values())
    if not r["shared"]:
        tot += sum(b.size for b in r["V"].values()) + sum(b.size for b in r["F"].values())
    tot += sum(b.size for l in range(r["q"] + 1) for b in r["S"][l])
    return int(tot)
