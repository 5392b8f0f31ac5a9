"""Cross-operator batches: every operator's result from one merged call must
match the oracle for that operator alone (bit-exact on integer
representations, within the 1e-12 * B bar otherwise), for mixed tree depths,
leaf sizes, ranks and per-operator vector counts (including nv = 0).  Graph
replays are checked against the eager result on every replay, with eager work
and synchronization between replays; the autotuned schedule is re-checked."""
import numpy as np
import pytest

import h2gen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def make_ops(seed):
    rng = np.random.default_rng(seed)
    bufs, kinds = [], []
    for i in range(5):  # integer random representations (exact)
        bufs.append(h2gen.random_rep(4000 + 10 * seed + i, q=int(rng.integers(0, 4)), max_leaf=8, max_rank=4))
        kinds.append("int")
    for i in range(6):  # built kernel matrices of uneven sizes, depths and ranks
        n = int(rng.integers(200, 3000))
        leaf = int(rng.integers(32, 65))
        p = int(rng.integers(3, 6))
        P = h2gen.points(n, 2, 5000 + 10 * seed + i)
        buf = h2gen.build(P, leaf=leaf, p=p, eta=0.7, kernel="exp", param=float(rng.uniform(0.05, 0.2)))
        bufs.append(np.array(buf.array, copy=True))
        kinds.append("float")
    return bufs, kinds


def inputs(refs, kinds, nv_max, seed):
    rng = np.random.default_rng(seed)
    Xs, Y0s, nvs, alphas, betas = [], [], [], [], []
    for i, (ref, kind) in enumerate(zip(refs, kinds)):
        nv = 0 if i == 2 else int(rng.integers(1, nv_max + 1))
        if kind == "int":
            X = rng.integers(-2, 3, size=(ref.n, max(nv, 1))).astype(np.float64)
            Y0 = rng.integers(-2, 3, size=(ref.n, max(nv, 1))).astype(np.float64)
            a, b = float(rng.choice([1.0, 2.0, 0.0])), float(rng.choice([0.0, -1.0, 3.0]))
        else:
            X = rng.standard_normal((ref.n, max(nv, 1)))
            Y0 = rng.standard_normal((ref.n, max(nv, 1)))
            a, b = 1.5, float(rng.choice([0.0, -0.5]))
        Xs.append(X[:, :nv] if nv else X[:, :0])
        Y0s.append(Y0[:, :nv] if nv else Y0[:, :0])
        nvs.append(nv)
        alphas.append(a)
        betas.append(b)
    return Xs, Y0s, nvs, alphas, betas


def to_dev(A):
    return torch.from_numpy(np.asfortranarray(A)).cuda() if A.shape[1] else None


def check(refs, kinds, Xs, Y0s, nvs, alphas, betas, Yd):
    for i, ref in enumerate(refs):
        if nvs[i] == 0:
            continue
        got = Yd[i].cpu().numpy()
        want = ref.gemv(Xs[i], alpha=alphas[i], beta=betas[i], Y=Y0s[i])
        if kinds[i] == "int":
            assert np.array_equal(got, want), i
        else:
            B = ref.gemv(Xs[i], alpha=alphas[i], beta=betas[i], Y=Y0s[i], absval=True)
            assert np.all(np.abs(got - want) <= 1e-12 * B), (i, np.max(np.abs(got - want) / B))


@pytest.mark.parametrize("nv_max", [4, 32])
def test_batch_matches_oracle(nv_max):
    from paper_2109_05451_amd import H2Batch
    bufs, kinds = make_ops(nv_max)
    refs = [oracle.Oracle(b) for b in bufs]
    batch = H2Batch(bufs, nv_max=nv_max)
    info = batch.info()
    assert info["count"] == len(bufs)
    Xs, Y0s, nvs, alphas, betas = inputs(refs, kinds, nv_max, 1)
    Xd = [to_dev(X) for X in Xs]
    Yd = [to_dev(Y) for Y in Y0s]
    batch.gemv(Xd, Yd, alphas, betas)
    torch.cuda.synchronize()
    check(refs, kinds, Xs, Y0s, nvs, alphas, betas, Yd)
    # autotuned shapes give the same results
    batch.tune(Xd, [to_dev(Y) for Y in Y0s], alphas, betas)
    Yd = [to_dev(Y) for Y in Y0s]
    batch.gemv(Xd, Yd, alphas, betas)
    torch.cuda.synchronize()
    check(refs, kinds, Xs, Y0s, nvs, alphas, betas, Yd)
    batch.close()


def test_batch_graph_replays():
    from paper_2109_05451_amd import H2Batch
    bufs, kinds = make_ops(7)
    refs = [oracle.Oracle(b) for b in bufs]
    batch = H2Batch(bufs, nv_max=16)
    stream = torch.cuda.Stream()
    eager = []
    inputs_list = [inputs(refs, kinds, 16, s) for s in range(3)]
    for Xs, Y0s, nvs, alphas, betas in inputs_list:
        Yd = [to_dev(Y) for Y in Y0s]
        Xd = [to_dev(X) for X in Xs]
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            batch.gemv(Xd, Yd, alphas, betas, stream=stream)
        stream.synchronize()
        eager.append([None if y is None else y.cpu().numpy() for y in Yd])
        check(refs, kinds, Xs, Y0s, nvs, alphas, betas, Yd)
    batch.graph(True)
    for rep in range(6):
        Xs, Y0s, nvs, alphas, betas = inputs_list[rep % 3]
        Yd = [to_dev(Y) for Y in Y0s]
        Xd = [to_dev(X) for X in Xs]
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            batch.gemv(Xd, Yd, alphas, betas, stream=stream)
        stream.synchronize()
        # eager work between replays
        junk = torch.randn(1000, 1000, device="cuda", dtype=torch.float64) @ torch.randn(
            1000, 1000, device="cuda", dtype=torch.float64)
        torch.cuda.synchronize()
        del junk
        for i, y in enumerate(Yd):
            if y is not None:
                assert np.array_equal(y.cpu().numpy(), eager[rep % 3][i]), (rep, i)
    batch.close()


def test_batch_per_operator_widths():
    """Operators bounded by 4, 16, 20, 40 and 64 vectors (three groups of
    widths 16, 32 and 48 or 64): each group's merged launches and workspace
    are separate; results are the oracle's (bit-exact on integer
    representations), and a call above an operator's bound is refused."""
    from paper_2109_05451_amd import H2Batch, H2Error
    bufs, kinds = make_ops(3)
    refs = [oracle.Oracle(b) for b in bufs]
    bounds = [4, 16, 20, 40, 64, 16, 4, 33, 48, 64, 1]
    batch = H2Batch(bufs, nv_max=bounds)
    assert batch.info()["launches"] > 10
    rng = np.random.default_rng(2)
    for rep in range(2):
        nvs = [int(rng.integers(0, b + 1)) for b in bounds]
        Xs, Y0s, alphas, betas = [], [], [], []
        for ref, kind, nv in zip(refs, kinds, nvs):
            if kind == "int":
                X = rng.integers(-2, 3, size=(ref.n, max(nv, 1))).astype(np.float64)
                Y0 = rng.integers(-2, 3, size=(ref.n, max(nv, 1))).astype(np.float64)
                a, b = 2.0, -1.0
            else:
                X = rng.standard_normal((ref.n, max(nv, 1)))
                Y0 = rng.standard_normal((ref.n, max(nv, 1)))
                a, b = 1.5, 0.0
            Xs.append(X[:, :nv]); Y0s.append(Y0[:, :nv]); alphas.append(a); betas.append(b)
        Xd = [to_dev(X) for X in Xs]
        Yd = [to_dev(Y) for Y in Y0s]
        if rep == 1:
            batch.tune(Xd, [to_dev(Y) for Y in Y0s], alphas, betas)
            # the plan description: one line per merged launch of every group
            # (each group's two permutations aside), with the tuned times
            info = batch.plan_info()
            groups = [l for l in info.splitlines() if l.startswith("group nvp=")]
            rows = [l for l in info.splitlines() if " rows=" in l]
            assert len(groups) >= 3 and info.startswith("schedule ")
            assert len(rows) == batch.info()["launches"] - 2 * len(groups)
            assert all(float(l.rsplit(" ", 1)[1].rstrip("ms")) > 0 for l in rows)
        batch.gemv(Xd, Yd, alphas, betas)
        torch.cuda.synchronize()
        check(refs, kinds, Xs, Y0s, nvs, alphas, betas, Yd)
    # an item above its operator's bound
    X = torch.zeros((refs[0].n, 5), dtype=torch.float64, device="cuda")
    Xd = [X if i == 0 else None for i in range(len(refs))]
    Yd = [torch.zeros_like(X) if i == 0 else None for i in range(len(refs))]
    with pytest.raises(H2Error):
        batch.gemv(Xd, Yd)
    batch.close()
