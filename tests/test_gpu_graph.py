"""Graph replay of single-operator products (h2_graph): every replay equals
the eager product bit for bit, with the input buffer refilled between
replays (X is read at replay time), eager work and synchronizations between
replays, a second set of buffers captured separately, retuning dropping the
graphs, both the streaming (1 vector) and multi-vector (20 vectors, FP64 and
FP32) paths, and schedules 0 and 3 (the latter forks a third stream inside
the capture); the eager products are the oracle's within the bars of
the other parity tests."""
import numpy as np
import pytest

import h2gen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def product(g, X, Y, nv, prec, stream, alpha=1.5, beta=-0.5):
    g.gemv_raw("N", alpha, X.data_ptr(), g.n, nv, beta, Y.data_ptr(), g.n, stream.cuda_stream, prec)


@pytest.mark.parametrize("schedule", [0, 3])
@pytest.mark.parametrize("nv,prec", [(1, "fp64"), (1, "fp32"), (20, "fp64"), (20, "fp32")])
def test_graph_replays_match_eager(nv, prec, schedule):
    from paper_2109_05451_amd import H2Operator
    buf = np.array(h2gen.build_config("c1_2d_4096").array, copy=True)
    ref = oracle.Oracle(buf)
    g = H2Operator(buf)
    g.prepare("fp32")
    g.set_schedule(prec, schedule)  # 3: a third stream forked into and joined back from the capture
    n = g.n
    stream = torch.cuda.Stream()
    rng = np.random.default_rng(nv)
    inputs = [rng.standard_normal((n, nv)) for _ in range(3)]
    Y0 = rng.standard_normal((n, nv))
    X = torch.empty((nv, n), dtype=torch.float64, device="cuda").t()
    Y = torch.empty((nv, n), dtype=torch.float64, device="cuda").t()
    # eager results
    eager = []
    for Xh in inputs:
        X.copy_(torch.from_numpy(Xh))
        Y.copy_(torch.from_numpy(Y0))
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            product(g, X, Y, nv, prec, stream)
        stream.synchronize()
        eager.append(Y.cpu().numpy())
        want = ref.gemv(Xh, alpha=1.5, beta=-0.5, Y=Y0)
        B = ref.gemv(Xh, alpha=1.5, beta=-0.5, Y=Y0, absval=True)
        tol = 1e-12 if prec == "fp64" else 2e-5
        assert np.all(np.abs(eager[-1] - want) <= tol * B)
    g.graph(True)
    for rep in range(7):
        k = rep % 3
        X.copy_(torch.from_numpy(inputs[k]))
        Y.copy_(torch.from_numpy(Y0))
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            product(g, X, Y, nv, prec, stream)  # rep 0 captures, the others replay
        stream.synchronize()
        junk = torch.randn(500, 500, dtype=torch.float64, device="cuda") @ torch.randn(
            500, 500, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        del junk
        assert np.array_equal(Y.cpu().numpy(), eager[k]), (rep, k)
    # other buffers: a second graph; the first still replays correctly
    X2 = torch.from_numpy(np.asfortranarray(inputs[1])).cuda()
    Y2 = torch.from_numpy(np.asfortranarray(Y0)).cuda()
    with torch.cuda.stream(stream):
        product(g, X2, Y2, nv, prec, stream)
    stream.synchronize()
    assert np.array_equal(Y2.cpu().numpy(), eager[1])
    # retuning drops the graphs; the next call captures afresh
    g.tune(64 if nv > 4 else 1, prec)
    g.set_schedule(prec, schedule)
    X.copy_(torch.from_numpy(inputs[2]))
    Y.copy_(torch.from_numpy(Y0))
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        product(g, X, Y, nv, prec, stream)
        product(g, X, Y2, nv, prec, stream, alpha=1.0, beta=0.0)
    stream.synchronize()
    assert np.array_equal(Y.cpu().numpy(), eager[2])
    g.graph(False)
    g.close()
    ref.close()
