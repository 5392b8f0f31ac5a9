"""The reduced-precision path (FP32 low-rank phases, FP64 dense near field and
final update) against the FP64 oracle.

Integer representations: every partial sum is an integer below 2^24, so the
FP32 path must be bit-exact too (this pins its indexing independently of
rounding).  Floating-point workloads: the low-rank data and arithmetic are
rounded to FP32 (unit roundoff 2^-24 ~ 6e-8); the elementwise bar is
2e-5 * B (B = oracle product in absolute values, which bounds every partial
sum), i.e. about 300 FP32 unit roundoffs, and the normwise relative error
is reported by the benchmark."""
import numpy as np
import pytest

import h2gen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL32 = 2e-5


def run(g, X, op="N", alpha=1.0, beta=0.0, Y0=None, precision="fp32"):
    Xd = torch.from_numpy(np.asfortranarray(X)).cuda()
    Yd = None if Y0 is None else torch.from_numpy(np.asfortranarray(Y0)).cuda()
    Y = g.gemv(Xd, op=op, alpha=alpha, beta=beta, Y=Yd, precision=precision)
    torch.cuda.synchronize()
    return Y.cpu().numpy()


@pytest.mark.parametrize("case", [dict(q=2), dict(q=3, separate=True), dict(q=3, max_children=1),
                                  dict(q=0), dict(q=4, max_children=2, p_adm=0.3)])
def test_fp32_integer_bitwise(case):
    from paper_2109_05451_amd import H2Operator
    for seed in range(3):
        buf = h2gen.random_rep(3000 + seed, **case)
        ref = oracle.Oracle(buf)
        g = H2Operator(buf)
        g.prepare("fp32")
        rng = np.random.default_rng(seed)
        for nv in (1, 4, 17, 64):
            X = rng.integers(-2, 3, size=(g.n, nv)).astype(np.float64)
            Y0 = rng.integers(-2, 3, size=(g.n, nv)).astype(np.float64)
            for op in "NT":
                want = ref.gemv(X, op=op, alpha=2.0, beta=-1.0, Y=Y0)
                got = run(g, X, op, 2.0, -1.0, Y0)
                assert np.array_equal(got, want), (case, seed, nv, op)
                if nv == 64 and op == "N":
                    # the balanced kernels, whose coupling launches gather
                    # from the FP32 copy of x^
                    g.tune_set("fp32", 8)
                    got = run(g, X, op, 2.0, -1.0, Y0)
                    g.tune_set("fp32", 64)
                    assert np.array_equal(got, want), (case, seed, nv, op, "kc 8")
        g.close()


@pytest.mark.parametrize("nv", [1, 3, 16, 40])
def test_fp32_small_config(nv):
    from paper_2109_05451_amd import H2Operator
    buf = h2gen.build_config("c1_2d_4096")
    ref = oracle.Oracle(buf.array)
    g = H2Operator(buf.array)
    X = h2gen.vectors(4096, nv, 2001)
    for op in "NT":
        want = ref.gemv(X, op=op)
        B = ref.gemv(X, op=op, absval=True)
        got = run(g, X, op)
        assert np.all(np.abs(got - want) <= TOL32 * B), np.max(np.abs(got - want) / B)
        rel = np.linalg.norm(got - want) / np.linalg.norm(want)
        assert 0 < rel < 1e-5, rel  # really reduced precision, and close
    g.close()


TOL16 = 5e-2  # BF16 data and staged vectors (unit roundoff 2^-9) along ~2(q+2) roundings, FP32 accumulation


def bf16_norm_bar(q):
    """Normwise bar for the BF16 path: an output sums terms along paths of
    about R = 2(q + 2) + 4 BF16 roundings (the bases and transfers of both
    sweeps, the stored vector trees at each level, the coupling blocks and
    the staged inputs), each a relative error of at most u = 2^-9 and, taken
    as independent and uniform, of RMS u / sqrt(3): the normwise error is
    about sqrt(R) u / sqrt(3).  Twice that is the bar (the elementwise
    TOL16 * B is the worst-case bound)."""
    return 2.0 * np.sqrt(2 * (q + 2) + 4) * 2.0 ** -9 / np.sqrt(3.0)


@pytest.mark.parametrize("cfg", ["c1", "laplace3d"])
@pytest.mark.parametrize("nv", [1, 16, 64])
def test_bf16(cfg, nv):
    from paper_2109_05451_amd import H2Operator, H2Error
    if cfg == "c1":
        buf = np.array(h2gen.build_config("c1_2d_4096").array, copy=True)
    else:  # rank 64 (4x4x4): the 16-byte BF16 fragment loads
        buf = np.array(h2gen.build(h2gen.points(6000, 3, 3), leaf=64, p=4, eta=0.7, kernel="laplace").array,
                       copy=True)
    ref = oracle.Oracle(buf)
    g = H2Operator(buf)
    X = h2gen.vectors(g.n, nv, 11)
    want = ref.gemv(X)
    B = ref.gemv(X, absval=True)
    got = run(g, X, "N", precision="bf16")
    assert np.all(np.abs(got - want) <= TOL16 * B), np.max(np.abs(got - want) / B)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert 0 < rel < bf16_norm_bar(g.stats()["depth"]), rel
    with pytest.raises(H2Error):
        run(g, X, "T", precision="bf16")
    g.close()


@pytest.mark.parametrize("cfg", ["c1", "laplace3d"])
def test_tune_keeps_results_bitwise(cfg):
    """h2_tune only picks chunk widths and grids; every candidate sums each
    output in the same order, so tuned results equal untuned ones bitwise."""
    from paper_2109_05451_amd import H2Operator
    if cfg == "c1":
        buf = np.array(h2gen.build_config("c1_2d_4096").array, copy=True)
    else:
        buf = np.array(h2gen.build(h2gen.points(6000, 3, 5), leaf=64, p=4, eta=0.7, kernel="laplace").array,
                       copy=True)
    ref = oracle.Oracle(buf)
    g = H2Operator(buf)
    X = h2gen.vectors(g.n, 40, 12)
    want = ref.gemv(X)
    B = ref.gemv(X, absval=True)
    for prec in ("fp64", "fp32", "bf16"):
        before = run(g, X, "N", precision=prec)
        g.tune(40, prec)
        after = run(g, X, "N", precision=prec)
        assert np.array_equal(before, after), prec
        if prec == "fp64":
            assert np.all(np.abs(after - want) <= 1e-12 * B)
    g.close()


# Grids of the multi-vector launches: one workgroup per row (0), persistent
# grids smaller than every launch's row count here (8, 24: each workgroup
# walks several rows, and with XCD-aware ranges each XCD's workgroups stride
# through their contiguous eighth), and one larger than most launches (1024:
# capped to one row per workgroup).
GRIDS = (0, 8, 24, 1024)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_launch_settings_bitwise(prec):
    """Every fixed setting of the multi-vector launches (chunk width or the
    pipelined kernel, the wave-per-row kernel, grid, XCD mapping, row order)
    gives bitwise the same
    product at 64 and 40 vectors, and the FP64 product is the oracle's to the
    1e-12 * B bar."""
    from paper_2109_05451_amd import H2Operator
    buf = np.array(h2gen.build(h2gen.points(5000, 2, 6), leaf=48, p=6, eta=0.7, kernel="exp").array, copy=True)
    ref = oracle.Oracle(buf)
    g = H2Operator(buf)
    # every launch of the plan has more rows than the small grids
    rows = [int(line.split("rows=")[1].split()[0]) for line in g.plan_info().splitlines() if "rows=" in line]
    assert min(rows) >= 1 and sum(r > 24 for r in rows) >= 4
    for nv in (64, 40):
        X = h2gen.vectors(g.n, nv, 13)
        base = run(g, X, "N", precision=prec)
        if prec == "fp64":
            want, B = ref.gemv(X), ref.gemv(X, absval=True)
            assert np.all(np.abs(base - want) <= 1e-12 * B)
        kcs = (64,) if prec == "bf16" else (0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 32, 64)
        for kc in kcs:
            for grid in GRIDS:
                for xcd in (False, True):
                    for tree in (0, 1):
                        g.tune_set(prec, kc, grid, xcd, tree)
                        got = run(g, X, "N", precision=prec)
                        assert np.array_equal(got, base), (prec, nv, kc, grid, xcd, tree)
    g.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("rank", [16, 36, 64])
def test_persistent_grids_walk_rows_against_oracle(prec, rank):
    """The 4096-point 2D operator (rank 16), and rank-36 (2D) and rank-64 (3D)
    operators of a few thousand points, with every launch on a persistent
    grid of 8 or 24 workgroups (several rows each), XCD-aware or not, in
    either row order: every output row against the oracle (bit-exact across
    settings; FP64 within 1e-12 * B, FP32 2e-5 * B, BF16 5e-2 * B)."""
    from paper_2109_05451_amd import H2Operator
    if rank == 16:
        buf = np.array(h2gen.build_config("c1_2d_4096").array, copy=True)
    elif rank == 36:
        buf = np.array(h2gen.build(h2gen.points(6000, 2, 16), leaf=64, p=6, eta=0.7, kernel="exp").array,
                       copy=True)
    else:
        buf = np.array(h2gen.build(h2gen.points(6000, 3, 17), leaf=64, p=4, eta=0.7, kernel="laplace").array,
                       copy=True)
    ref = oracle.Oracle(buf)
    g = H2Operator(buf)
    X = h2gen.vectors(g.n, 64, 14)
    want, B = ref.gemv(X), ref.gemv(X, absval=True)
    tol = {"fp64": 1e-12, "fp32": TOL32, "bf16": TOL16}[prec]
    kcs = (64,) if prec == "bf16" else (0, 5, 8, 9, 10, 11, 12, 32, 64)
    first = None
    for kc in kcs:
        for grid in (8, 24):
            for xcd in (False, True):
                for tree in (0, 1):
                    g.tune_set(prec, kc, grid, xcd, tree)
                    got = run(g, X, "N", precision=prec)
                    if first is None:
                        first = got
                        assert np.all(np.abs(got - want) <= tol * B), (prec, rank, np.max(np.abs(got - want) / B))
                    assert np.array_equal(got, first), (prec, rank, kc, grid, xcd, tree)
    g.close()
    ref.close()
