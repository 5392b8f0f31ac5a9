"""GPU recompression (h2_compress) and export (h2_export) against the oracle.

What is unique is compared: the ranks per level (integers, exact), and the
compressed operator as a matrix (its product with seeded vectors through the
product oracle, on the GPU's exported representation and on the oracle's).
Bases and coupling blocks themselves are not unique (signs, rotations among
the padding), so they are not compared entry by entry.  The GPU carries Gram
matrices where the oracle carries QR factors, so the two compressed matrices
agree to about eps / tau^2 relative; the tolerance is 1e-8 of the oracle's
absolute-value bound.  Every case is first checked to keep its singular values
clear of the threshold (relative gap above 1e-6), so that rounding cannot
decide a kept count.
"""
import numpy as np
import pytest

import h2gen
import oracle
from oracle import h2_compress as hc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-8


def cases():
    out = []
    for seed, kw in [(31, dict(q=3, max_children=2)), (32, dict(q=3, max_children=2, separate=True)),
                     (33, dict(q=2, max_children=3, p_adm=0.6)), (34, dict(q=4, max_children=2, separate=True))]:
        out.append((f"rand{seed}", np.array(h2gen.random_rep(seed, integer=False, max_leaf=6, max_rank=4,
                                                               allow_empty=False, **kw), copy=True)))
    out.append(("exp2d", np.array(h2gen.build(h2gen.points(3000, 2, 41), leaf=32, p=6, eta=0.7,
                                              kernel="exp").array, copy=True)))
    out.append(("lap3d", np.array(h2gen.build(h2gen.points(2500, 3, 42), leaf=40, p=3, eta=0.7,
                                              kernel="laplace").array, copy=True)))
    return out


CASES = cases()


def product(buf, X):
    o = oracle.Oracle(buf)
    y, B = o.gemv(X), o.gemv(X, absval=True)
    o.close()
    return y, B


def clear_of_threshold(info, tau):
    for side in ("row", "col"):
        eps = tau * info[f"sigma_ref_{side}"]
        for s in info[f"sigma_{side}"].values():
            if s.size and np.any(np.abs(s - eps) <= 1e-6 * max(eps, 1e-300)):
                return False
    return True


@pytest.mark.parametrize("name,buf", CASES, ids=[c[0] for c in CASES])
def test_export_roundtrip(name, buf):
    from paper_2109_05451_amd import H2Operator
    g = H2Operator(buf)
    got = g.export()
    want = hc.write(hc.read(buf))  # the same representation without points
    if hc.read(buf)["points"] is not None:
        r = hc.read(buf)
        r["points"] = None
        want = hc.write(r)
    assert np.array_equal(got, want)
    g.close()


@pytest.mark.parametrize("tau", [1e-2, 1e-3, 1e-5])
@pytest.mark.parametrize("name,buf", CASES, ids=[c[0] for c in CASES])
def test_compress_matches_oracle(name, buf, tau):
    from paper_2109_05451_amd import H2Operator
    cb, info = hc.compress(buf, tau)
    if not clear_of_threshold(info, tau):
        pytest.skip("a singular value sits at the threshold for this case")
    g = H2Operator(buf)
    gc, ginfo = g.compress(tau)
    kr, kc = gc.ranks()
    assert np.array_equal(kr, info["krow"]) and np.array_equal(kc, info["kcol"]), (kr, info["krow"])
    assert np.isclose(ginfo["sigma_ref_row"], info["sigma_ref_row"], rtol=1e-10)
    assert ginfo["lowrank_entries_after"] == hc.lowrank_entries(cb)
    n = g.n
    X = h2gen.vectors(n, 3, 7)
    want, B = product(cb, X)
    exported = gc.export()
    got, _ = product(exported, X)
    assert np.all(np.abs(got - want) <= TOL * B), np.max(np.abs(got - want) / B)
    # the compressed handle's own product equals its exported representation's
    Y = gc.gemv(torch.from_numpy(np.asfortranarray(X)).cuda())
    torch.cuda.synchronize()
    Yg = Y.cpu().numpy()
    assert np.all(np.abs(Yg - got) <= 1e-12 * product(exported, X)[1])
    # the original handle is untouched
    Y0 = g.gemv(torch.from_numpy(np.asfortranarray(X)).cuda()).cpu().numpy()
    y0, B0 = product(buf, X)
    assert np.all(np.abs(Y0 - y0) <= 1e-12 * B0)
    gc.close()
    g.close()


@pytest.mark.parametrize("name,buf", CASES, ids=[c[0] for c in CASES])
def test_compress_tau_zero_keeps_matrix(name, buf):
    """tau = 0 keeps every direction whose squared singular value is above
    rounding: the matrix is kept to about sqrt(eps) of the low-rank part."""
    from paper_2109_05451_amd import H2Operator
    g = H2Operator(buf)
    gc, _ = g.compress(0.0)
    X = h2gen.vectors(g.n, 2, 8)
    y0, B = product(buf, X)
    y1, _ = product(gc.export(), X)
    assert np.all(np.abs(y1 - y0) <= 1e-6 * B)
    gc.close()
    g.close()


def test_compress_twice_and_reject_bad_tau():
    from paper_2109_05451_amd import H2Error, H2Operator
    buf = CASES[4][1]
    g = H2Operator(buf)
    with pytest.raises(H2Error):
        g.compress(1.0)
    with pytest.raises(H2Error):
        g.compress(-1e-3)
    a, _ = g.compress(1e-3)
    b, _ = a.compress(1e-3)  # compressing an orthogonal, truncated operator again
    X = h2gen.vectors(g.n, 2, 9)
    ya, B = product(a.export(), X)
    yb, _ = product(b.export(), X)
    assert np.all(np.abs(yb - ya) <= 1e-2 * B)
    assert b.ranks()[0].sum() <= a.ranks()[0].sum()
    for h in (a, b, g):
        h.close()
