"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bar: bit-exact where every partial sum is an integer (any summation order
gives the same bits); otherwise elementwise
    |Y_gpu - Y_oracle| <= 1e-12 * B,
where B is the oracle's product with every entry, input, alpha and beta
replaced by its absolute value (it bounds every partial sum of any evaluation
order, so 1e-12 * B is a rounding allowance of about 9000 unit roundoffs),
plus the normwise relative error <= 1e-12 that the FP64 path is held to.
"""
import numpy as np
import pytest

import h2gen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


def dev(a):
    t = torch.from_numpy(np.asfortranarray(a, dtype=np.float64))
    return t.cuda()


def operator(buf):
    from paper_2109_05451_amd import H2Operator
    return H2Operator(buf, device=0)


def run(op_obj, X, op="N", alpha=1.0, beta=0.0, Y0=None):
    Y = op_obj.gemv(dev(X), op=op, alpha=alpha, beta=beta, Y=None if Y0 is None else dev(Y0))
    torch.cuda.synchronize()
    return Y.cpu().numpy()


def assert_close(got, want, bound, what=""):
    diff = np.abs(got - want)
    bad = diff > TOL * bound
    assert not bad.any(), f"{what}: {bad.sum()} entries beyond 1e-12*B, worst {np.max(diff / np.maximum(bound, 1e-300)):.3e}"
    nw = np.linalg.norm(want)
    if nw > 0:
        assert np.linalg.norm(got - want) <= TOL * nw, f"{what}: normwise {np.linalg.norm(got - want) / nw:.3e}"


INT_CASES = [
    dict(q=0), dict(q=1), dict(q=2), dict(q=3), dict(q=3, max_children=1), dict(q=2, separate=False),
    dict(q=4, max_children=2, p_adm=0.3), dict(q=2, p_adm=0.0), dict(q=2, p_adm=1.0),
    dict(q=3, allow_empty=False, max_leaf=9, max_rank=5),
]


@pytest.mark.parametrize("case", range(len(INT_CASES)))
def test_integer_representations_bitwise(case):
    for seed in range(3):
        buf = h2gen.random_rep(1000 + 10 * case + seed, **INT_CASES[case])
        ref = oracle.Oracle(buf)
        g = operator(buf)
        rng = np.random.default_rng(seed)
        for nv in (1, 3, 9):
            X = rng.integers(-2, 3, size=(g.n, nv)).astype(np.float64)
            Y0 = rng.integers(-2, 3, size=(g.n, nv)).astype(np.float64)
            for op in "NT":
                for alpha, beta in ((1.0, 0.0), (2.0, -1.0), (0.0, 3.0)):
                    want = ref.gemv(X, op=op, alpha=alpha, beta=beta, Y=Y0)
                    got = run(g, X, op, alpha, beta, Y0)
                    assert np.array_equal(got, want), (case, seed, nv, op, alpha, beta)
        g.close()


@pytest.mark.parametrize("nv", [1, 2, 7, 16, 33, 64, 65])
def test_small_config_parity(nv):
    """2D, n = 4096, leaf 64, 4x4 Chebyshev, eta 0.7, exp(-r/0.1)."""
    buf = h2gen.build_config("c1_2d_4096")
    ref = oracle.Oracle(buf.array)
    g = operator(buf.array)
    X = h2gen.vectors(4096, nv, 2001)
    Y0 = h2gen.vectors(4096, nv, 77)
    for op in "NT":
        for alpha, beta in ((1.0, 0.0), (1.5, -0.5)):
            want = ref.gemv(X, op=op, alpha=alpha, beta=beta, Y=Y0)
            B = ref.gemv(X, op=op, alpha=alpha, beta=beta, Y=Y0, absval=True)
            got = run(g, X, op, alpha, beta, Y0)
            assert_close(got, want, B, f"nv={nv} op={op} a={alpha} b={beta}")
    g.close()


@pytest.mark.parametrize("seed", range(6))
def test_float_representations(seed):
    """Non-symmetric random representations with ragged leaves and ranks."""
    buf = h2gen.random_rep(2000 + seed, q=3 + seed % 2, max_children=3, max_leaf=12, max_rank=7,
                           integer=False, p_adm=0.35)
    ref = oracle.Oracle(buf)
    g = operator(buf)
    X = np.random.default_rng(seed).standard_normal((g.n, 5))
    for op in "NT":
        want = ref.gemv(X, op=op)
        got = run(g, X, op)
        assert_close(got, want, ref.gemv(X, op=op, absval=True), f"seed={seed} op={op}")
    g.close()


@pytest.mark.parametrize("nv", [3, 20])
@pytest.mark.parametrize("kind,dim,p", [("laplace", 3, 3), ("exp", 2, 6), ("gauss", 2, 5)])
def test_built_operators(kind, dim, p, nv):
    """Odd ranks and leaf sizes (27, 47): exercises the masked MFMA tiles."""
    P = h2gen.points(6000, dim, 5 + dim)
    buf = h2gen.build(P, leaf=48, p=p, eta=0.7, kernel=kind, param=0.15)
    ref = oracle.Oracle(buf.array)
    g = operator(buf.array)
    X = h2gen.vectors(6000, nv, 9)
    for op in "NT":
        want = ref.gemv(X, op=op)
        got = run(g, X, op)
        assert_close(got, want, ref.gemv(X, op=op, absval=True), f"{kind} op={op}")
    g.close()


def test_edge_cases():
    buf = h2gen.random_rep(3, q=3, integer=False)
    ref = oracle.Oracle(buf)
    g = operator(buf)
    n = g.n
    X = np.random.default_rng(0).standard_normal((n, 4))
    # nv = 0: no work, no error
    g.gemv_raw("N", 1.0, 0, n, 0, 0.0, 0, n)
    # beta = 0 must not read Y (NaN-safe)
    Ynan = np.full((n, 4), np.nan)
    got = run(g, X, "N", 1.0, 0.0, Ynan)
    assert_close(got, ref.gemv(X), ref.gemv(X, absval=True), "beta=0")
    # alpha = 0: Y <- beta Y, X not read (pass a NULL X)
    Y0 = np.random.default_rng(1).standard_normal((n, 4))
    Yd = dev(Y0)
    g.gemv_raw("N", 0.0, 0, n, 4, 2.0, Yd.data_ptr(), n)
    torch.cuda.synchronize()
    assert np.array_equal(Yd.cpu().numpy(), 2.0 * Y0)
    # leading dimensions larger than n
    ld = n + 13
    Xb = torch.zeros((4, ld), dtype=torch.float64, device="cuda")
    Xb[:, :n] = torch.from_numpy(X.T.copy()).cuda()
    Yb = torch.full((4, ld), 7.0, dtype=torch.float64, device="cuda")
    g.gemv_raw("T", 1.0, Xb.data_ptr(), ld, 4, 0.0, Yb.data_ptr(), ld)
    torch.cuda.synchronize()
    got = Yb.cpu().numpy()[:, :n].T
    assert_close(got, ref.gemv(X, op="T"), ref.gemv(X, op="T", absval=True), "ld > n")
    assert np.all(Yb.cpu().numpy()[:, n:] == 7.0)  # padding untouched
    # argument errors are reported, not crashed on
    from paper_2109_05451_amd import H2Error
    with pytest.raises(H2Error):
        g.gemv_raw("X", 1.0, Xb.data_ptr(), ld, 4, 0.0, Yb.data_ptr(), ld)
    with pytest.raises(H2Error):
        g.gemv_raw("N", 1.0, Xb.data_ptr(), n - 1, 4, 0.0, Yb.data_ptr(), ld)
    with pytest.raises(H2Error):
        g.gemv_raw("N", 1.0, Xb.data_ptr(), ld, 4, 0.0, Xb.data_ptr(), ld)  # overlap
    g.close()


def test_single_point_and_single_leaf():
    for n in (1, 2, 50):
        P = h2gen.points(n, 2, n)
        buf = h2gen.build(P, leaf=64, p=3, eta=0.7, kernel="exp")
        ref = oracle.Oracle(buf.array)
        g = operator(buf.array)
        X = h2gen.vectors(n, 2, 1)
        got = run(g, X)
        assert_close(got, ref.gemv(X), ref.gemv(X, absval=True), f"n={n}")
        g.close()


def test_deterministic():
    buf = h2gen.build_config("c1_2d_4096")
    g = operator(buf.array)
    X = h2gen.vectors(4096, 16, 5)
    a = run(g, X)
    b = run(g, X)
    assert np.array_equal(a, b)
    g.close()


def test_reserve_and_stats():
    buf = h2gen.build_config("c1_2d_4096")
    g = operator(buf.array)
    st = g.stats()
    assert st["n"] == 4096 and st["depth"] == 6 and st["nleaves"] == 64
    assert st["entries_U"] == 4096 * 16 and st["shared_basis"] == 1
    g.reserve(64)
    st2 = g.stats()
    assert st2["device_bytes"] > st["device_bytes"]
    # algorithmic work (every stored entry read once; x^, y^ written and read once)
    entries = sum(st["entries_" + k] for k in "UVEFSD")
    assert st["alg_flops_per_vector"] == 2 * entries + st["n"]
    assert st["alg_bytes_matrix"] == 8 * entries
    assert st["alg_bytes_per_vector"] == 8 * (2 * st["n"] + 4 * st["tree_rows"])
    # per-level structure adds up to the totals
    ls = g.level_stats()
    assert len(ls) == st["depth"] + 1
    assert [x["nodes"] for x in ls] == [2 ** l for l in range(st["depth"] + 1)]
    assert all(x["krow"] == x["kcol"] == 16 for x in ls)
    assert sum(x["coupling_blocks"] for x in ls) == st["ncoupling"]
    assert sum(x["entries_S"] for x in ls) == st["entries_S"]
    assert sum(x["entries_E"] for x in ls) == st["entries_E"] == sum(x["entries_F"] for x in ls)
    assert max(x["csp"] for x in ls) == st["csp"]
    assert ls[0]["coupling_blocks"] == 0 and ls[0]["entries_E"] == 0
    g.close()
