"""Parity at full size for the 3D workload: N = 2^19 points uniform in [0,1]^3,
leaf 64, kernel 1/(4 pi r) with zero diagonal, 4x4x4 Chebyshev (rank 64),
eta 0.7, nv = 64 (the MFMA path), tuned as bench.py tunes it, in FP64 and in
the BF16 and FP32 variants.

Every output row of two vector columns is compared with the oracle's
product of those columns alone (columns are independent: pinned in the
oracle's tests), and 32 sampled rows of all 64 columns with the oracle's
rows computed one by one.  Bars of the small tests: 1e-12 * B (FP64),
2e-5 * B (FP32), 5e-2 * B (BF16), B the oracle's product in absolute
values; normwise, the BF16 results also stay within twice the statistical
estimate sqrt(R) u / sqrt(3) of R = 2(q + 2) + 4 roundings of unit roundoff
2^-9 (1.3e-2 at q = 13)."""
import numpy as np
import pytest

import h2gen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 2e-5, "bf16": 5e-2}


def test_full_size_3d_every_row_of_two_columns_and_sampled_rows():
    buf = h2gen.build_config("c3_3d_512k")
    from paper_2109_05451_amd import H2Operator
    g = H2Operator(buf.array, device=0)
    n, nv = g.n, 64
    Xh = h2gen.vectors(n, nv, 2003)
    X = torch.from_numpy(np.asfortranarray(Xh)).cuda()
    Y = torch.empty((nv, n), dtype=torch.float64, device="cuda").t()
    stream = torch.cuda.current_stream().cuda_stream
    g.reserve(nv)
    cols = [3, 50]
    rows = np.unique(np.concatenate([[0, n - 1], np.random.default_rng(3).integers(0, n, 30)]))
    got_cols, got_rows = {}, {}
    for prec in ("fp64", "bf16", "fp32"):
        if prec != "fp64":
            g.prepare(prec)
        g.tune(nv, prec, stream)
        g.gemv_raw("N", 1.0, X.data_ptr(), n, nv, 0.0, Y.data_ptr(), n, stream, prec)
        torch.cuda.synchronize()
        assert bool(torch.isfinite(Y).all().item()), prec
        got_cols[prec] = Y[:, cols].cpu().numpy()
        got_rows[prec] = Y[torch.from_numpy(rows).cuda()].cpu().numpy()
    q = g.stats()["depth"]
    g.close()
    del X, Y
    ref = oracle.Oracle(buf.array)
    Xc = np.asfortranarray(Xh[:, cols])
    checks = [(got_cols, ref.gemv(Xc), ref.gemv(Xc, absval=True), "all rows of two columns"),
              (got_rows, ref.gemv_rows(rows, Xh), ref.gemv_rows(rows, Xh, absval=True), "sampled rows")]
    for got, want, B, what in checks:
        for prec, tol in TOL.items():
            diff = np.abs(got[prec] - want)
            assert np.all(diff <= tol * B), (what, prec, float(np.max(diff / B)))
            assert np.linalg.norm(got[prec] - want) <= tol * np.linalg.norm(want), (what, prec)
        bar16 = 2.0 * np.sqrt(2 * (q + 2) + 4) * 2.0 ** -9 / np.sqrt(3.0)
        rel16 = np.linalg.norm(got["bf16"] - want) / np.linalg.norm(want)
        assert rel16 <= bar16, (what, rel16, bar16)
    ref.close()
