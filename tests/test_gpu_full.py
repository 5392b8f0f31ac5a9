"""Parity at the benchmark's full size, in the launch configuration bench.py
times: 2D, N = 2^20, leaf 64, 6x6 Chebyshev (rank 36), eta 0.7, exp(-r/0.1),
nv = 1 and nv = 16.  The oracle computes sampled output rows one by one
(h2o_gemv_rows: the whole column upsweep, then only the coupling rows on the
sampled leaves' root paths), and the GPU result is compared on those rows
to the same 1e-12 bar as the small parity tests."""
import numpy as np
import pytest

import h2gen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c2():
    buf = h2gen.build_config("c2_2d_1m")
    from paper_2109_05451_amd import H2Operator
    g = H2Operator(buf.array, device=0)
    ref = oracle.Oracle(buf.array)
    yield buf, g, ref
    g.close()
    ref.close()


@pytest.mark.parametrize("nv", [1, 16])
def test_full_size_sampled_rows(c2, nv):
    buf, g, ref = c2
    n = g.n
    Xh = h2gen.vectors(n, nv, 2002)
    X = torch.from_numpy(np.asfortranarray(Xh)).cuda()
    Y = torch.empty((nv, n), dtype=torch.float64, device="cuda").t()
    g.reserve(nv)
    g.gemv_raw("N", 1.0, X.data_ptr(), n, nv, 0.0, Y.data_ptr(), n, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    got = Y.cpu().numpy()
    rows = np.unique(np.concatenate([[0, n - 1, n // 2], np.random.default_rng(nv).integers(0, n, 61)]))
    want = ref.gemv_rows(rows, Xh)
    B = ref.gemv_rows(rows, Xh, absval=True)
    diff = np.abs(got[rows] - want)
    assert np.all(diff <= 1e-12 * B), np.max(diff / B)
    assert np.linalg.norm(got[rows] - want) <= 1e-12 * np.linalg.norm(want)
    # property at every row: finite output
    assert np.all(np.isfinite(got))
