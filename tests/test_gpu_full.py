"""Parity at the benchmark's full size, in the launch configuration bench.py
times (multi-vector launches tuned with h2_tune first): 2D, N = 2^20, leaf 64,
6x6 Chebyshev (rank 36), eta 0.7, exp(-r/0.1), nv = 1, 16 and 64, in FP64 and
in the FP32 variant.  The oracle computes sampled output rows one by one
(h2o_gemv_rows: the whole column upsweep, then only the coupling rows on the
sampled leaves' root paths), and the GPU result is compared on those rows to
the same bars as the small tests: 1e-12 * B for FP64, 2e-5 * B for FP32 (B:
the oracle's product in absolute values)."""
import numpy as np
import pytest

import h2gen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 2e-5}


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


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nv", [1, 16, 64])
def test_full_size_sampled_rows(c2, nv, prec):
    buf, g, ref, cache = c2
    n = g.n
    Xh = h2gen.vectors(n, nv, 2002)
    X = torch.from_numpy(np.asfortranarray(Xh)).cuda()
    Y = torch.empty((nv, n), dtype=torch.float64, device="cuda").t()
    stream = torch.cuda.current_stream().cuda_stream
    g.reserve(nv)
    if prec != "fp64":
        g.prepare(prec)
    g.tune(nv, prec, stream)
    g.gemv_raw("N", 1.0, X.data_ptr(), n, nv, 0.0, Y.data_ptr(), n, stream, prec)
    torch.cuda.synchronize()
    got = Y.cpu().numpy()
    rows = np.unique(np.concatenate([[0, n - 1, n // 2], np.random.default_rng(nv).integers(0, n, 61)]))
    if nv not in cache:
        cache[nv] = (ref.gemv_rows(rows, Xh), ref.gemv_rows(rows, Xh, absval=True))
    want, B = cache[nv]
    diff = np.abs(got[rows] - want)
    assert np.all(diff <= TOL[prec] * B), np.max(diff / B)
    rel = np.linalg.norm(got[rows] - want) / np.linalg.norm(want)
    assert rel <= TOL[prec]
    if prec == "fp32":
        assert rel > 0  # really the reduced-precision path
    # property at every row: finite output
    assert np.all(np.isfinite(got))
