"""The fragment-ordered matrix copies of the wave-row kernels
(h2_set_fragment_order, made by h2_tune too: FP64 for every op-'N' row, FP32
for the low-rank rows).  Wave-row launches that read them get the same MFMA
operands in the same order as from the column-major data, so the products
must be bitwise those of a handle without the copies under the same fixed
kernel settings: a wave per row and a wave per 16-vector tile (each also in
its form compiled for five waves per SIMD), one workgroup per row and a
persistent grid smaller than the row count, with and without the XCD-aware
row ranges.  The operators cover ranks whose row
tiles are ragged (25 = 16 + 9, 27 = 16 + 11) or whole (16, 64), odd leaf
sizes, and column counts that are not multiples of eight (the copy's
column-major tail).  FP64 results are the oracle's within 1e-12 * B."""
import numpy as np
import pytest

import h2gen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

OPS = {
    "2d_k25_leaf37": dict(n=5000, dim=2, seed=61, leaf=37, p=5, kernel="exp"),
    "2d_k16_leaf64": dict(n=4096, dim=2, seed=62, leaf=64, p=4, kernel="exp"),
    "3d_k27_leaf41": dict(n=5000, dim=3, seed=63, leaf=41, p=3, kernel="laplace"),
    "3d_k64_leaf64": dict(n=4000, dim=3, seed=64, leaf=64, p=4, kernel="laplace"),
}


def run(g, X, prec):
    Y = g.gemv(torch.from_numpy(np.asfortranarray(X)).cuda(), precision=prec)
    torch.cuda.synchronize()
    return Y.cpu().numpy()


@pytest.mark.parametrize("name", sorted(OPS))
def test_fragment_order_bitwise(name):
    from paper_2109_05451_amd import H2Operator
    o = OPS[name]
    buf = np.array(h2gen.build(h2gen.points(o["n"], o["dim"], o["seed"]), leaf=o["leaf"], p=o["p"], eta=0.7,
                               kernel=o["kernel"]).array, copy=True)
    ref = oracle.Oracle(buf)
    tuned, plain = H2Operator(buf), H2Operator(buf)
    for nv in (16, 40, 64):
        X = h2gen.vectors(tuned.n, nv, 70 + nv)
        want, B = ref.gemv(X), ref.gemv(X, absval=True)
        for prec in ("fp64", "fp32"):
            tuned.tune(nv, prec)  # keeps the copies only where a launch reads them
            tuned.set_fragment_order(prec, True)
            plain.set_fragment_order(prec, False)
            for g in (tuned, plain):
                g.set_sweeps(prec, False)  # per-level launches: every phase on the row kernels
                g.set_schedule(prec, 0)
            kcs = (9, 10, 11, 12) if nv > 16 else (9, 11)
            for kc in kcs:
                for grid in (0, 24):
                    for xcd in (False, True):
                        tuned.tune_set(prec, kc, grid, xcd)
                        plain.tune_set(prec, kc, grid, xcd)
                        a, b = run(tuned, X, prec), run(plain, X, prec)
                        assert np.array_equal(a, b), (name, nv, prec, kc, grid, xcd)
                        if prec == "fp64":
                            assert np.all(np.abs(a - want) <= 1e-12 * B), (name, nv, kc, grid, xcd)
    before = tuned.stats()["device_bytes"]
    assert before > plain.stats()["device_bytes"]  # the copies are accounted
    for prec in ("fp64", "fp32"):
        tuned.set_fragment_order(prec, False)  # no launch reads them: freed
    assert tuned.stats()["device_bytes"] < before
    tuned.close()
    plain.close()
    ref.close()
