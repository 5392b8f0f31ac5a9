"""The fused sweeps of the multi-vector path (each workgroup runs several
levels of one subtree: upsweep bottom-up, downsweep top-down ending with the
leaf expansion) against the per-level launches and the oracle.

Integer representations (entries and inputs in {-2..2}) keep every partial
sum an integer below 2^53: fused, per-level and oracle agree bit for bit, on
trees of any arity (one to three children), empty leaves, depth 0 to 6,
shared and separate bases with different row and column ranks, and vector
counts that pad to every tile width.  On built kernel matrices the two
launch forms are bitwise equal (same summation order) and within the
1e-12 * B bar of the oracle (FP64) or 2e-5 * B (FP32)."""
import numpy as np
import pytest

import h2gen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def run(g, X, precision="fp64", alpha=1.0, beta=0.0, Y0=None):
    Xd = torch.from_numpy(np.asfortranarray(X)).cuda()
    Yd = None if Y0 is None else torch.from_numpy(np.asfortranarray(Y0)).cuda()
    Y = g.gemv(Xd, alpha=alpha, beta=beta, Y=Yd, precision=precision)
    torch.cuda.synchronize()
    return Y.cpu().numpy()


CASES = [dict(q=0), dict(q=1), dict(q=3, max_children=3), dict(q=4, max_children=2, p_adm=0.3),
         dict(q=5, max_children=2, separate=False), dict(q=6, max_children=2, max_leaf=5, max_rank=3),
         dict(q=3, max_children=1), dict(q=4, max_children=3, allow_empty=True)]


@pytest.mark.parametrize("ci", range(len(CASES)))
def test_fused_sweeps_integer_bitwise(ci):
    from paper_2109_05451_amd import H2Operator
    case = CASES[ci]
    for seed in range(2):
        buf = h2gen.random_rep(7100 + 10 * ci + seed, **case)
        ref = oracle.Oracle(buf)
        g = H2Operator(buf)
        g.prepare("fp32")
        assert "tree workgroups" in g.plan_info()
        rng = np.random.default_rng(seed)
        for nv in (5, 17, 40, 64):
            X = rng.integers(-2, 3, size=(g.n, nv)).astype(np.float64)
            Y0 = rng.integers(-2, 3, size=(g.n, nv)).astype(np.float64)
            want = ref.gemv(X, alpha=2.0, beta=-1.0, Y=Y0)
            for prec in ("fp64", "fp32"):
                got = {}
                for fused in (True, False):
                    g.set_sweeps(prec, fused)
                    got[fused] = run(g, X, prec, 2.0, -1.0, Y0)
                assert np.array_equal(got[True], want), (case, seed, nv, prec)
                assert np.array_equal(got[False], got[True]), (case, seed, nv, prec)
        g.close()
        ref.close()


@pytest.mark.parametrize("cfg", ["2d_rank36", "3d_rank64", "2d_rank16"])
def test_fused_sweeps_built_operators(cfg):
    from paper_2109_05451_amd import H2Operator
    if cfg == "2d_rank36":
        buf = h2gen.build(h2gen.points(20000, 2, 31), leaf=64, p=6, eta=0.7, kernel="exp").array
    elif cfg == "3d_rank64":
        buf = h2gen.build(h2gen.points(12000, 3, 32), leaf=64, p=4, eta=0.7, kernel="laplace").array
    else:
        buf = h2gen.build_config("c1_2d_4096").array
    buf = np.array(buf, copy=True)
    ref = oracle.Oracle(buf)
    g = H2Operator(buf)
    g.prepare("fp32")
    last = None
    for nv in (16, 48, 64):
        X = h2gen.vectors(g.n, nv, 40 + nv)
        want, B = ref.gemv(X), ref.gemv(X, absval=True)
        for prec, tol in (("fp64", 1e-12), ("fp32", 2e-5)):
            got = {}
            for fused in (True, False):
                g.set_sweeps(prec, fused)
                got[fused] = run(g, X, prec)
            assert np.array_equal(got[True], got[False]), (cfg, nv, prec)
            assert np.all(np.abs(got[True] - want) <= tol * B), (cfg, nv, prec)
            if prec == "fp64":
                last = got[True]
    # the tuner keeps whichever form is faster; the bits do not change
    g.tune(64)
    assert "sweeps" in g.plan_info()
    assert np.array_equal(run(g, X), last)
    g.close()
    ref.close()


def test_fused_sweeps_refused_for_rank_above_64():
    from paper_2109_05451_amd import H2Error, H2Operator
    buf = h2gen.random_rep(124, q=2, max_children=2, max_leaf=80, ranks=([70] * 3, [70] * 3), p_adm=0.3,
                           integer=True, int_range=1, allow_empty=False)
    g = H2Operator(buf)
    with pytest.raises(H2Error):
        g.set_sweeps("fp64", True)
    g.set_sweeps("fp64", False)
    ref = oracle.Oracle(buf)
    X = np.random.default_rng(1).integers(-2, 3, size=(g.n, 20)).astype(np.float64)
    assert np.array_equal(run(g, X), ref.gemv(X))
    g.close()
