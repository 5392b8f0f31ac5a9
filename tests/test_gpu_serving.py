"""Serving loop: requests for operators of different sizes, nv in
{1, 4, 16, 64}, FP64 and FP32 classes are admitted, fused and run
concurrently; every result must equal the same request computed alone (and
the oracle) within its precision's bar: 1e-12 * B for FP64, 2e-5 * B for
FP32 (B = the oracle's product in absolute values).

What makes it a serving loop and not a queue is asserted too: requests that
wait while a slot is busy are fused into fewer calls than requests, calls on
different slots are in flight at once, and requests keep arriving (from a
submitter thread) while earlier ones run.  Inputs still being produced on
the submitter's stream when they are submitted are read only after that
work (the request's event), with no synchronization by the caller."""
import threading
import time

import numpy as np
import pytest

import h2gen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def operators():
    from paper_2109_05451_amd import H2Operator
    bufs = [h2gen.build_config("c1_2d_4096").array,
            h2gen.build(h2gen.points(3000, 3, 4), leaf=48, p=3, eta=0.7, kernel="laplace").array,
            h2gen.random_rep(77, q=4, max_children=2, max_leaf=16, max_rank=6, integer=False),
            # one to two milliseconds per 64-vector call: calls overlap with arrivals
            h2gen.build(h2gen.points(1 << 18, 2, 8), leaf=64, p=5, eta=0.7, kernel="exp", param=0.1).array]
    bufs = [np.array(b, copy=True) for b in bufs]
    ops = [H2Operator(b) for b in bufs]
    for o in ops:
        o.prepare("fp32")
    refs = [oracle.Oracle(b) for b in bufs]
    return ops, refs


@pytest.fixture(scope="module")
def served():
    ops, refs = operators()
    yield ops, refs
    for o in ops:
        o.close()
    for r in refs:
        r.close()


def check(ops, refs, op, prec, Xh, X, Y):
    got = Y.cpu().numpy()
    solo = ops[op].gemv(X, precision=prec)
    torch.cuda.synchronize()
    want = refs[op].gemv(Xh)
    B = refs[op].gemv(Xh, absval=True)
    tol = 1e-12 if prec == "fp64" else 2e-5
    assert np.all(np.abs(got - want) <= tol * B), (op, prec, np.max(np.abs(got - want) / B))
    assert np.all(np.abs(got - solo.cpu().numpy()) <= 2 * tol * B), (op, prec)


def test_burst_is_fused_and_overlapped(served):
    from paper_2109_05451_amd import H2Server
    ops, refs = served
    server = H2Server(ops, slots=2, budget_bytes=1 << 30, max_fuse_nv=64)
    rng = np.random.default_rng(0)
    reqs = []
    for k in range(40):
        op = int(rng.integers(0, 4))
        nv = int(rng.choice([1, 4, 16, 64]))
        prec = "fp64" if k % 2 == 0 else "fp32"
        Xh = rng.standard_normal((ops[op].n, nv))
        X = torch.from_numpy(np.asfortranarray(Xh)).cuda()
        reqs.append((op, prec, Xh, X))
    torch.cuda.synchronize()
    ids = [server.submit(op, X, prec) for (op, prec, Xh, X) in reqs]
    outs = [server.wait(i) for i in ids]
    st = server.stats()
    server.close()
    assert st["completed"] == 40 and st["submitted"] == 40
    assert st["calls"] < st["submitted"], st          # waiting requests were fused
    assert st["max_inflight_calls"] >= 2, st          # both slots held calls at once
    assert st["vectors"] == sum(X.shape[1] for (_, _, _, X) in reqs)
    assert st["alg_bytes"] > 0 and st["alg_flops"] > 0
    for (op, prec, Xh, X), (Y, lat) in zip(reqs, outs):
        assert lat > 0
        check(ops, refs, op, prec, Xh, X, Y)


def test_staggered_arrivals_join_running_work(served):
    """Two 64-vector requests on the 2^18-point operator occupy both slots;
    a submitter thread then sends small requests every 0.1 ms.  They arrive
    while those calls run, queue, and are fused into later calls that
    overlap with each other."""
    from paper_2109_05451_amd import H2Server
    ops, refs = served
    server = H2Server(ops, slots=2, budget_bytes=1 << 30, max_fuse_nv=64)
    rng = np.random.default_rng(1)
    reqs = []
    for k in range(34):
        if k < 2:
            op, nv, prec = 3, 64, "fp64"
        else:
            op = 3 if k % 3 else int(rng.integers(0, 3))
            nv = int(rng.choice([1, 4, 16]))
            prec = "fp64" if k % 4 else "fp32"
        Xh = rng.standard_normal((ops[op].n, nv))
        reqs.append((op, prec, Xh, torch.from_numpy(np.asfortranarray(Xh)).cuda()))
    torch.cuda.synchronize()
    ids = [None] * len(reqs)
    outstanding = []

    def submitter():
        for k, (op, prec, Xh, X) in enumerate(reqs):
            ids[k] = server.submit(op, X, prec)
            st = server.stats()
            outstanding.append(st["submitted"] - st["completed"])
            if k >= 1:
                time.sleep(1e-4)

    th = threading.Thread(target=submitter)
    th.start()
    outs = []
    for k in range(len(reqs)):
        while ids[k] is None:
            time.sleep(1e-4)
        outs.append(server.wait(ids[k]))
    th.join()
    st = server.stats()
    server.close()
    assert st["completed"] == len(reqs)
    assert max(outstanding) >= 3             # arrivals found earlier requests unfinished
    assert st["calls"] < st["submitted"], st  # queued arrivals joined later calls
    assert st["max_inflight_calls"] >= 2, st
    for (op, prec, Xh, X), (Y, lat) in zip(reqs, outs):
        check(ops, refs, op, prec, Xh, X, Y)


def test_input_still_in_production_is_awaited(served):
    """X is produced on the current stream behind a long matrix product and
    handed over row-major (the binding makes the column-major copy on that
    stream); nothing synchronizes before submit."""
    from paper_2109_05451_amd import H2Server
    ops, refs = served
    server = H2Server(ops, slots=2, budget_bytes=1 << 30, max_fuse_nv=64)
    op = 3
    n = ops[op].n
    rng = np.random.default_rng(2)
    Xh = rng.standard_normal((n, 5))
    base = torch.from_numpy(np.ascontiguousarray(Xh)).cuda()  # row-major n x 5
    big = torch.ones((6144, 6144), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    busy = big @ big                               # tens of ms on the current stream
    X = (base * 2.0 + busy[0, 0] * 0.0)            # ready only after the product
    rid = server.submit(op, X, "fp64")
    Y, _ = server.wait(rid)
    server.close()
    check(ops, refs, op, "fp64", 2.0 * Xh, torch.from_numpy(np.asfortranarray(2.0 * Xh)).cuda(), Y)


def test_unprepared_precision_is_refused():
    from paper_2109_05451_amd import H2Error, H2Operator, H2Server
    g = H2Operator(np.array(h2gen.build_config("c1_2d_4096").array, copy=True))
    server = H2Server([g], slots=1, budget_bytes=0, max_fuse_nv=16)
    st = server.stats()
    assert 0 < st["budget_bytes"] <= st["hbm_free_at_create"]
    X = torch.zeros((g.n, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(H2Error):
        server.submit(0, X, "fp32")
    Y, _ = server.wait(server.submit(0, X, "fp64"))
    assert torch.count_nonzero(Y).item() == 0
    server.close()
    g.close()
