"""The batched workload at its own scale, as bench.py runs it: 256 independent
2D operators, N = round(2^U(12,16)), leaf U{32..64}, Chebyshev p in {4,5,6},
exp(-r/l) with l ~ U[0.05, 0.2], eta 0.7, nv ~ U{1..32} (each operator's
bound, so two vector widths: 16 and 32), merged level by level, autotuned,
replayed from a captured HIP graph.  For every operator,
sampled output rows (both ends and six seeded ones) of every vector are
compared with the oracle's rows of that operator alone, computed one by one
(h2o_gemv_rows), to the FP64 bar 1e-12 * B; every output is finite."""
import numpy as np
import pytest

import h2gen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_256_operators_every_operator_sampled_rows():
    import bench
    from paper_2109_05451_amd import H2Batch
    specs = bench.batch_ops(256)
    bufs = [h2gen.build(h2gen.points(sp["n"], 2, sp["seed_pts"]), sp["leaf"], sp["p"], 0.7, "exp", sp["ell"])
            for sp in specs]
    batch = H2Batch([b.array for b in bufs], nv_max=[sp["nv"] for sp in specs])
    assert batch.info()["count"] == 256
    Xh = [h2gen.vectors(sp["n"], sp["nv"], sp["seed_vec"]) for sp in specs]
    Xs = [torch.from_numpy(np.asfortranarray(x)).cuda() for x in Xh]
    Ys = [torch.empty((sp["nv"], sp["n"]), dtype=torch.float64, device="cuda").t() for sp in specs]
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    batch.tune(Xs, Ys, stream=stream)
    batch.graph(True)
    with torch.cuda.stream(stream):
        for _ in range(3):  # capture, then replays
            for y in Ys:
                y.fill_(float("nan"))
            batch.gemv(Xs, Ys, stream=stream)
    stream.synchronize()
    batch.close()
    for i, (sp, b) in enumerate(zip(specs, bufs)):
        Y = Ys[i]
        assert bool(torch.isfinite(Y).all().item()), i
        n = sp["n"]
        rows = np.unique(np.concatenate([[0, n - 1], np.random.default_rng(i).integers(0, n, 6)]))
        got = Y[torch.from_numpy(rows).cuda()].cpu().numpy()
        ref = oracle.Oracle(b.array)
        want = ref.gemv_rows(rows, Xh[i])
        B = ref.gemv_rows(rows, Xh[i], absval=True)
        ref.close()
        assert np.all(np.abs(got - want) <= 1e-12 * B), (i, sp, float(np.max(np.abs(got - want) / B)))
