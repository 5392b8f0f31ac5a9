"""Pins of the recompression oracle (Section 5 of the paper) against things
other than itself:

* brute force on tiny representations, from the dense low-rank matrix: the
  singular values of every node's reweighting factor equal those of the block
  row its basis must represent (own and ancestors' coupling blocks, plus the
  block columns for a shared basis), which pins orthogonalization and the
  reweighting downsweep; every new explicit basis spans the leading singular
  subspace of that block row projected on its children's new bases, the kept
  counts follow the threshold rule, and the compressed low-rank matrix is the
  two-sided projection of the original (the projection step);
* closed forms: tau = 0 reproduces the operator; an operator inflated from
  rank r to a larger stored rank (same matrix) compresses back to rank <= r
  and the same matrix;
* orthogonality of the new explicit bases; the error of a compressed kernel
  matrix falls with tau and stays within a small multiple of tau.
"""
import numpy as np
import pytest

import brute
import h2gen
import oracle
from h2gen import fmt
from oracle import h2_compress as hc


def reps():
    out = []
    for seed, kw in [(11, dict(q=2, max_children=3)), (12, dict(q=3, max_children=2, separate=True)),
                     (13, dict(q=3, max_children=2)), (14, dict(q=2, max_children=3, separate=True, p_adm=0.6)),
                     (15, dict(q=1, max_children=3))]:
        out.append(np.array(h2gen.random_rep(seed, integer=False, max_leaf=5, max_rank=3, allow_empty=False,
                                             **kw), copy=True))
    return out


def product(buf, X):
    o = oracle.Oracle(buf)
    y = o.gemv(X)
    B = o.gemv(X, absval=True)
    o.close()
    return y, B


@pytest.mark.parametrize("idx", range(5))
def test_roundtrip_reader_writer(idx):
    buf = reps()[idx]
    assert np.array_equal(hc.write(hc.read(buf)), buf)


@pytest.mark.parametrize("idx", range(5))
def test_orthogonalize_keeps_matrix_and_orthonormalizes(idx):
    buf = reps()[idx]
    rep = hc.orthogonalize(hc.read(buf))
    ob = hc.write(rep)
    X = np.random.default_rng(idx).standard_normal((hc.read(buf)["n"], 3))
    y0, B = product(buf, X)
    y1, _ = product(ob, X)
    assert np.all(np.abs(y1 - y0) <= 1e-12 * B + 1e-14)
    r = fmt.parse(ob)
    for which in ("U", "V"):
        Bh = brute.explicit_bases(r, which)
        for c, Q in Bh.items():
            G = Q.T @ Q
            # orthonormal columns, or zero columns where a stack had too few rows
            d = np.diag(G)
            assert np.allclose(G, np.diag(d), atol=1e-12)
            assert np.all((np.abs(d - 1) < 1e-12) | (np.abs(d) < 1e-12))


def _sv(A):
    return np.linalg.svd(A, compute_uv=False) if A.size else np.zeros(0)


@pytest.mark.parametrize("idx", range(5))
def test_weights_match_block_rows(idx):
    """sigma(R_i) = sigma(block row of node i) for every node (brute force)."""
    buf = reps()[idx]
    Alr, r = brute.dense_tree_order(buf, include_dense=False)
    rep = hc.orthogonalize(hc.read(buf))
    shared = rep["shared"]
    for side in (("row",) if shared else ("row", "col")):
        W = hc.weights(rep, side)
        for i in range(r["nnodes"]):
            G = brute.block_row(Alr, r, i, rows=side == "row" or shared, cols=side == "col" or shared)
            s_bf = _sv(G)
            s_or = _sv(W[i])
            scale = max(1.0, s_bf[0] if s_bf.size else 0.0)
            k = min(s_bf.size, s_or.size)
            assert np.allclose(s_or[:k], s_bf[:k], atol=1e-11 * scale), (side, i)
            assert np.all(s_bf[k:] < 1e-11 * scale) and np.all(s_or[k:] < 1e-11 * scale)


def _projector(Q):
    return Q @ np.linalg.pinv(Q) if Q.size else np.zeros((Q.shape[0], Q.shape[0]))


@pytest.mark.parametrize("idx", range(5))
@pytest.mark.parametrize("tau", [0.05, 0.3])
def test_truncation_and_projection_by_brute_force(idx, tau):
    buf = reps()[idx]
    Alr, r = brute.dense_tree_order(buf, include_dense=False)
    cb, info = hc.compress(buf, tau)
    rc = fmt.parse(cb)
    shared = not (r["flags"] & 1)
    q, lp = r["q"], r["level_ptr"]
    proj = {}
    for side in (("row",) if shared else ("row", "col")):
        newb = brute.explicit_bases(rc, "U" if side == "row" else "V")
        rows, cols = side == "row" or shared, side == "col" or shared
        G = {i: brute.block_row(Alr, r, i, rows=rows, cols=cols) for i in range(r["nnodes"])}
        sref = max((_sv(G[t])[0] for t in range(int(lp[q]), int(lp[q + 1])) if G[t].size), default=0.0)
        assert np.isclose(sref, info["sigma_ref_row" if side == "row" else "sigma_ref_col"], rtol=1e-12, atol=0)
        eps = tau * sref
        counts = info["count_row" if side == "row" else "count_col"]
        P = {}
        for l in range(q, -1, -1):
            for i in range(int(lp[l]), int(lp[l + 1])):
                if l == q:
                    Gi = G[i]
                else:
                    kids = [c for c in range(int(lp[l + 1]), int(lp[l + 2])) if r["parent"][c] == i]
                    lo_i = r["lo"][i]
                    Pc = np.zeros((G[i].shape[0],) * 2)
                    for c in kids:
                        a, b = r["lo"][c] - lo_i, r["hi"][c] - lo_i
                        Pc[a:b, a:b] = P[c]
                    Gi = Pc @ G[i]
                if Gi.size:
                    Wl, s, _ = np.linalg.svd(Gi, full_matrices=False)
                else:
                    Wl, s = np.zeros((Gi.shape[0], 0)), np.zeros(0)
                # the case is clear of the threshold
                assert np.all(np.abs(s - eps) > 1e-6 * max(sref, 1e-300)), (side, i)
                c_bf = int(np.sum(s > eps))
                assert counts[i] == c_bf, (side, i)
                P[i] = Wl[:, :c_bf] @ Wl[:, :c_bf].T
                assert np.allclose(_projector(newb[i]), P[i], atol=1e-9), (side, i)
        proj[side] = P
    Pr = proj["row"]
    Pc = proj["row"] if shared else proj["col"]
    want = np.zeros_like(Alr)
    lo, hi = r["lo"], r["hi"]
    for _, t, s in brute.coupling_blocks(r):
        want[lo[t]:hi[t], lo[s]:hi[s]] = Pr[t] @ Alr[lo[t]:hi[t], lo[s]:hi[s]] @ Pc[s]
    got, _ = brute.dense_tree_order(cb, include_dense=False)
    assert np.allclose(got, want, atol=1e-10 * max(1.0, np.abs(Alr).max()))
    # dense blocks are untouched
    assert np.array_equal(rc["D"], r["D"])


@pytest.mark.parametrize("idx", range(5))
def test_tau_zero_reproduces_operator(idx):
    buf = reps()[idx]
    cb, _ = hc.compress(buf, 0.0)
    X = np.random.default_rng(7).standard_normal((hc.read(buf)["n"], 2))
    y0, B = product(buf, X)
    y1, _ = product(cb, X)
    assert np.all(np.abs(y1 - y0) <= 1e-11 * B + 1e-13)


def inflate(buf, kk, seed):
    """Same matrix stored with rank kk per level: U_t -> U_t Phi_t with a
    random full-row-rank Phi (r x kk) and right inverse Psi (Phi Psi = I);
    E_c -> Psi_c E_c Phi_p, S_ts -> Psi_t S_ts Psi_s^T."""
    rep = hc.read(buf)
    rng = np.random.default_rng(seed)
    q, lp = rep["q"], rep["level_ptr"]

    def maps(k):
        Phi, Psi = {}, {}
        for l in range(q + 1):
            for c in range(int(lp[l]), int(lp[l + 1])):
                r_ = int(k[l])
                A = rng.standard_normal((r_, kk))
                Phi[c] = A
                Psi[c] = np.linalg.pinv(A)
        return Phi, Psi

    out = dict(rep)
    Phr, Psr = maps(rep["krow"])
    if rep["shared"]:
        Phc, Psc = Phr, Psr
    else:
        Phc, Psc = maps(rep["kcol"])
    out["U"] = {t: U @ Phr[t] for t, U in rep["U"].items()}
    out["E"] = {c: Psr[c] @ E @ Phr[int(rep["parent"][c])] for c, E in rep["E"].items()}
    if not rep["shared"]:
        out["V"] = {t: V @ Phc[t] for t, V in rep["V"].items()}
        out["F"] = {c: Psc[c] @ F @ Phc[int(rep["parent"][c])] for c, F in rep["F"].items()}
    out["S"] = [[Psr[t] @ blk @ Psc[s].T for (t, s), blk in zip(hc._blocks(rep, l), rep["S"][l])]
                for l in range(q + 1)]
    out["krow"] = np.full(q + 1, kk, np.int64)
    out["kcol"] = np.full(q + 1, kk, np.int64)
    return hc.write(out), rep


@pytest.mark.parametrize("idx", range(5))
def test_inflated_rank_is_recovered(idx):
    buf = reps()[idx]
    big, rep = inflate(buf, 6, idx)
    X = np.random.default_rng(idx).standard_normal((rep["n"], 2))
    y0, B = product(buf, X)
    yb, _ = product(big, X)
    assert np.all(np.abs(yb - y0) <= 1e-10 * B + 1e-12)  # the inflation kept the matrix
    cb, info = hc.compress(big, 1e-9)
    assert np.all(info["krow"] <= rep["krow"]) and np.all(info["kcol"] <= rep["kcol"])
    y1, _ = product(cb, X)
    assert np.all(np.abs(y1 - y0) <= 1e-7 * B + 1e-9)


def test_kernel_matrix_error_follows_tau():
    """Exponential kernel in 2D: the compressed product's relative error stays
    below 2 tau (the threshold is relative to the largest block row; the
    truncations of the levels add up) and falls with tau; the low-rank storage
    shrinks."""
    buf = np.array(h2gen.build(h2gen.points(3000, 2, 21), leaf=32, p=6, eta=0.7, kernel="exp").array, copy=True)
    X = h2gen.vectors(3000, 2, 22)
    y0, _ = product(buf, X)
    n0 = hc.lowrank_entries(buf)
    errs, sizes = [], []
    for tau in (1e-2, 1e-3, 1e-4, 1e-5):
        cb, info = hc.compress(buf, tau)
        y1, _ = product(cb, X)
        errs.append(np.linalg.norm(y1 - y0) / np.linalg.norm(y0))
        sizes.append(hc.lowrank_entries(cb))
        assert errs[-1] < 2 * tau, (tau, errs[-1])
    assert all(a > b for a, b in zip(errs, errs[1:]))
    assert all(a < b for a, b in zip(sizes, sizes[1:])) and sizes[-1] < n0


def test_compressed_bases_orthonormal_on_kernel_matrix():
    buf = np.array(h2gen.build(h2gen.points(1500, 3, 23), leaf=32, p=3, eta=0.7, kernel="laplace").array,
                   copy=True)
    cb, info = hc.compress(buf, 1e-3)
    r = fmt.parse(cb)
    for c, Q in brute.explicit_bases(r, "U").items():
        G = Q.T @ Q
        d = np.diag(G)
        assert np.allclose(G, np.diag(d), atol=1e-12)
        assert np.all((np.abs(d - 1) < 1e-12) | (np.abs(d) < 1e-12))
