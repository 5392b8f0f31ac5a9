"""Serving loop: a burst of mixed requests (operators of different sizes,
nv in {1, 4, 16, 64}, FP64 and FP32 classes) is admitted, fused and run
concurrently; every result must equal the same request computed alone (and
the oracle) within its precision's bar: 1e-12 * B for FP64, 2e-5 * B for
FP32 (B = the oracle's product in absolute values)."""
import numpy as np
import pytest

import h2gen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_mixed_requests_match_solo_results():
    from paper_2109_05451_amd import H2Operator, H2Server
    bufs = [h2gen.build_config("c1_2d_4096").array,
            h2gen.build(h2gen.points(3000, 3, 4), leaf=48, p=3, eta=0.7, kernel="laplace").array,
            h2gen.random_rep(77, q=4, max_children=2, max_leaf=16, max_rank=6, integer=False)]
    bufs = [np.array(b, copy=True) for b in bufs]
    ops = [H2Operator(b) for b in bufs]
    refs = [oracle.Oracle(b) for b in bufs]
    server = H2Server(ops, slots=2, budget_bytes=64 << 20, max_fuse_nv=64)
    rng = np.random.default_rng(0)
    reqs = []
    for k in range(40):
        op = int(rng.integers(0, 3))
        nv = int(rng.choice([1, 4, 16, 64]))
        prec = "fp64" if k % 2 == 0 else "fp32"
        Xh = rng.standard_normal((ops[op].n, nv))
        X = torch.from_numpy(np.asfortranarray(Xh)).cuda()
        reqs.append((op, prec, Xh, X))
    torch.cuda.synchronize()
    ids = [server.submit(op, X, prec) for (op, prec, Xh, X) in reqs]
    outs = [server.wait(i) for i in ids]
    st = server.stats()
    assert st["completed"] == 40 and st["submitted"] == 40
    assert st["calls"] <= 40
    for (op, prec, Xh, X), (Y, lat) in zip(reqs, outs):
        assert lat > 0
        got = Y.cpu().numpy()
        solo = ops[op].gemv(X, precision=prec)
        torch.cuda.synchronize()
        want = refs[op].gemv(Xh)
        B = refs[op].gemv(Xh, absval=True)
        tol = 1e-12 if prec == "fp64" else 2e-5
        assert np.all(np.abs(got - want) <= tol * B), (op, prec, np.max(np.abs(got - want) / B))
        assert np.all(np.abs(got - solo.cpu().numpy()) <= 2 * tol * B)
    server.close()
    for o in ops:
        o.close()
