"""Parity at the benchmark's full size, in the launch configuration bench.py
times (multi-vector launches tuned with h2_tune first): 2D, N = 2^20, leaf 64,
6x6 Chebyshev (rank 36), eta 0.7, exp(-r/0.1), nv = 1, 16 and 64, in FP64 and
in the FP32 variant.

* nv = 1: every one of the 2^20 output rows against the oracle's whole
  product.
* nv = 16, 64: every output row of four of the vector columns against the
  oracle's product of those columns alone (columns are independent: pinned
  in the oracle's tests), plus 64 sampled rows of all columns, which the
  oracle computes one by one (h2o_gemv_rows: the whole column upsweep, then
  only the coupling rows on the sampled leaves' root paths).

Bars as in the small tests: 1e-12 * B for FP64, 2e-5 * B for FP32 (B: the
oracle's product in absolute values, which bounds every partial sum)."""
import numpy as np
import pytest

import h2gen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 2e-5}
COLS = {16: [0, 5, 11, 15], 64: [0, 17, 40, 63]}


@pytest.fixture(scope="module")
def c2():
    buf = h2gen.build_config("c2_2d_1m")
    from paper_2109_05451_amd import H2Operator
    g = H2Operator(buf.array, device=0)
    ref = oracle.Oracle(buf.array)
    cache = {}
    yield buf, g, ref, cache
    g.close()
    ref.close()


def gpu_product(g, Xh, nv, prec):
    n = g.n
    X = torch.from_numpy(np.asfortranarray(Xh)).cuda()
    Y = torch.empty((nv, n), dtype=torch.float64, device="cuda").t()
    stream = torch.cuda.current_stream().cuda_stream
    g.reserve(nv)
    if prec != "fp64":
        g.prepare(prec)
    g.tune(nv, prec, stream)
    g.gemv_raw("N", 1.0, X.data_ptr(), n, nv, 0.0, Y.data_ptr(), n, stream, prec)
    torch.cuda.synchronize()
    return Y.cpu().numpy()


def check(got, want, B, prec, what):
    diff = np.abs(got - want)
    assert np.all(diff <= TOL[prec] * B), (what, float(np.max(diff / B)))
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert rel <= TOL[prec], (what, rel)
    if prec == "fp32":
        assert rel > 0, what  # really the reduced-precision path
    return rel


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_full_size_every_row_nv1(c2, prec):
    buf, g, ref, cache = c2
    Xh = h2gen.vectors(g.n, 1, 2002)
    got = gpu_product(g, Xh, 1, prec)
    if "nv1" not in cache:
        cache["nv1"] = (ref.gemv(Xh), ref.gemv(Xh, absval=True))
    want, B = cache["nv1"]
    check(got, want, B, prec, "all rows, nv=1")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nv", [16, 64])
def test_full_size_every_row_of_four_columns(c2, nv, prec):
    buf, g, ref, cache = c2
    n = g.n
    Xh = h2gen.vectors(n, nv, 2002)
    got = gpu_product(g, Xh, nv, prec)
    assert np.all(np.isfinite(got))
    cols = COLS[nv]
    key = ("cols", nv)
    if key not in cache:
        Xc = np.asfortranarray(Xh[:, cols])
        cache[key] = (ref.gemv(Xc), ref.gemv(Xc, absval=True))
    want, B = cache[key]
    check(got[:, cols], want, B, prec, f"all rows of columns {cols}, nv={nv}")
    rows = np.unique(np.concatenate([[0, n - 1, n // 2], np.random.default_rng(nv).integers(0, n, 61)]))
    key = ("rows", nv)
    if key not in cache:
        cache[key] = (ref.gemv_rows(rows, Xh), ref.gemv_rows(rows, Xh, absval=True))
    want, B = cache[key]
    check(got[rows], want, B, prec, f"sampled rows, all {nv} columns")
