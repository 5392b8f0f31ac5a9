"""The largest supported sizes and the fallback for rows wider than the LDS
block tables, bit-exact against the oracle.

Integer data (entries in {-1, 0, 1} or {-2..2}, inputs in {-2..2}) keep every
partial sum an integer below 2^53, so any summation order gives the same bits.
Ranks and leaf sizes of 256 exercise the row kernels' largest tile counts (16
row tiles, four per wave on the MFMA path) and the transposed kernel's LDS
passes; rows of more than 512 blocks go to the wide-row kernel (and keep the
product on the streaming path)."""
import numpy as np
import pytest

import h2gen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def run(g, X, op, alpha, beta, Y0):
    Xd = torch.from_numpy(np.asfortranarray(X)).cuda()
    Yd = torch.from_numpy(np.asfortranarray(Y0)).cuda()
    Y = g.gemv(Xd, op=op, alpha=alpha, beta=beta, Y=Yd)
    torch.cuda.synchronize()
    return Y.cpu().numpy()


def check_bitwise(buf, nvs, tune_nv=None):
    from paper_2109_05451_amd import H2Operator
    ref = oracle.Oracle(buf)
    g = H2Operator(buf)
    rng = np.random.default_rng(5)
    for nv in nvs:
        X = rng.integers(-2, 3, size=(g.n, nv)).astype(np.float64)
        Y0 = rng.integers(-2, 3, size=(g.n, nv)).astype(np.float64)
        for op in "NT":
            for alpha, beta in ((1.0, 0.0), (2.0, -1.0)):
                want = ref.gemv(X, op=op, alpha=alpha, beta=beta, Y=Y0)
                got = run(g, X, op, alpha, beta, Y0)
                assert np.array_equal(got, want), (nv, op, alpha, beta)
    if tune_nv:
        X = rng.integers(-2, 3, size=(g.n, tune_nv)).astype(np.float64)
        Y0 = np.zeros((g.n, tune_nv))
        g.tune(tune_nv)
        assert np.array_equal(run(g, X, "N", 1.0, 0.0, Y0), ref.gemv(X))
    info = g.plan_info()
    g.close()
    ref.close()
    return info


@pytest.mark.parametrize("seed", [124, 141])
def test_rank_and_leaf_256(seed):
    buf = h2gen.random_rep(seed, q=2, max_children=3, max_leaf=256, ranks=([256] * 3, [256] * 3), p_adm=0.3,
                           integer=True, int_range=1, allow_empty=False)
    check_bitwise(buf, (1, 3, 17, 64), tune_nv=64)


def test_rows_wider_than_the_block_table():
    buf = h2gen.random_rep(92, q=10, max_children=3, max_leaf=2, max_rank=2, p_adm=0.05, integer=True)
    info = check_bitwise(buf, (1, 3, 9))
    assert "kind=2" in info  # some dense rows (945 blocks) took the wide-row kernel


@pytest.mark.parametrize("seed", [7, 8])
def test_ranks_33_to_36_every_kernel(seed):
    """Rows of 33-36 outputs take the 4x4x4 MFMA for their last four rows in
    the balanced kernels' four- and five-workgroup forms.  Ranks 33-36 per
    level (separate row and column bases) and leaves of 1-40 points mix such
    rows with shorter and longer ones in one launch; at 64 vectors every
    kernel setting must give the oracle's integer result bit for bit."""
    from paper_2109_05451_amd import H2Operator
    buf = h2gen.random_rep(seed, q=3, max_children=3, max_leaf=40, ranks=([34, 33, 35, 36], [36, 35, 33, 34]),
                           p_adm=0.4, integer=True, int_range=1, allow_empty=False)
    ref = oracle.Oracle(buf)
    g = H2Operator(buf)
    rng = np.random.default_rng(seed)
    X = rng.integers(-2, 3, size=(g.n, 64)).astype(np.float64)
    Y0 = rng.integers(-2, 3, size=(g.n, 64)).astype(np.float64)
    want = ref.gemv(X, op="N", alpha=2.0, beta=-1.0, Y=Y0)
    for kc in (0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 32, 64):
        for grid in (0, 8, 24, 1024):  # 8, 24: persistent grids walking several rows each
            for xcd in ((False, True) if grid in (8, 24) else (False,)):
                g.tune_set("fp64", kc, grid, xcd, 0)
                got = run(g, X, "N", 2.0, -1.0, Y0)
                assert np.array_equal(got, want), (seed, kc, grid, xcd)
    g.close()
    ref.close()
