"""h2_gemv_noalloc (the product on the library's fixed per-GPU scratch array,
for callers that cannot allocate) against h2_gemv on the same handle and
against the oracle, through the C ABI.

Two calls in a row, the second with a smaller input, so the second runs on
scratch that still holds the first call's contents.  Integer representations
keep every partial sum an integer below 2^53: both entry points and the
oracle must agree bit for bit.  The floating-point operator is held to the
FP64 bar of the other parity tests (1e-12 * B, B the oracle's product in
absolute values) against the oracle, and to 2e-12 * B against h2_gemv (the
two entry points may take different pass widths, so different chunkings of a
row's columns)."""
import ctypes

import numpy as np
import pytest

import h2gen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def call(lib_fn, g, X, Y, op, alpha, beta):
    n, nv = X.shape
    rc = lib_fn(g._h, op.encode(), alpha, X.data_ptr(), n, nv, beta, Y.data_ptr(), n,
                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, rc


def both(g, Xh, Y0h, op, alpha, beta):
    from paper_2109_05451_amd import load_library
    lib = load_library()
    X = torch.from_numpy(np.asfortranarray(Xh)).cuda()
    Y_na = torch.from_numpy(np.asfortranarray(Y0h)).cuda()
    Y_al = Y_na.clone()
    assert Y_na.stride(0) == Y_al.stride(0) == 1
    assert Y_na.shape[1] == 1 or Y_al.stride(1) == Y_na.stride(1) == g.n
    call(lib.h2_gemv_noalloc, g, X, Y_na, op, alpha, beta)
    call(lib.h2_gemv, g, X, Y_al, op, alpha, beta)
    torch.cuda.synchronize()
    return Y_na.cpu().numpy(), Y_al.cpu().numpy()


def test_noalloc_matches_gemv_two_calls_second_smaller():
    from paper_2109_05451_amd import H2Operator
    rng = np.random.default_rng(21)
    # first call: the 4096-point 2D operator, 6 vectors (passes of 4 and 2)
    big = np.array(h2gen.build_config("c1_2d_4096").array, copy=True)
    ref_big = oracle.Oracle(big)
    g_big = H2Operator(big)
    X = rng.standard_normal((g_big.n, 6))
    Y0 = rng.standard_normal((g_big.n, 6))
    for op in "NT":
        na, al = both(g_big, X, Y0, op, 1.5, -0.5)
        want = ref_big.gemv(X, op=op, alpha=1.5, beta=-0.5, Y=Y0)
        B = ref_big.gemv(X, op=op, alpha=1.5, beta=-0.5, Y=Y0, absval=True)
        assert np.all(np.abs(na - want) <= 1e-12 * B), (op, np.max(np.abs(na - want) / B))
        assert np.all(np.abs(na - al) <= 2e-12 * B), op
    # second call: a smaller integer representation, fewer vectors
    small = h2gen.random_rep(33, q=3, max_children=3, max_leaf=6, max_rank=4, p_adm=0.4, integer=True)
    ref_small = oracle.Oracle(small)
    g_small = H2Operator(small)
    assert g_small.n < g_big.n
    Xi = rng.integers(-2, 3, size=(g_small.n, 3)).astype(np.float64)
    Yi = rng.integers(-2, 3, size=(g_small.n, 3)).astype(np.float64)
    for op in "NT":
        for alpha, beta in ((1.0, 0.0), (2.0, -1.0), (0.0, 3.0)):
            na, al = both(g_small, Xi, Yi, op, alpha, beta)
            want = ref_small.gemv(Xi, op=op, alpha=alpha, beta=beta, Y=Yi)
            assert np.array_equal(na, want), (op, alpha, beta)
            assert np.array_equal(na, al), (op, alpha, beta)
    g_big.close()
    g_small.close()


def test_noalloc_narrow_passes_2d_2e20():
    """A 2^20-point operator (leaf 32, 3x3 Chebyshev): one column of scratch
    is 8 (2 n + 2 H) = 26 MB, so the fixed array takes passes of two columns
    where h2_gemv takes four; against h2_gemv and the oracle, then a call
    with one column (the same pass width on both sides: bitwise equal)."""
    from paper_2109_05451_amd import H2Operator
    buf = h2gen.build(h2gen.points(1 << 20, 2, 41), leaf=32, p=3, eta=0.7, kernel="exp", param=0.1)
    ref = oracle.Oracle(buf.array)
    g = H2Operator(buf.array)
    st = g.stats()
    per = 8 * (2 * st["n"] + 2 * st["tree_rows"])
    assert (64 << 20) // per == 2
    rng = np.random.default_rng(3)
    for nv in (3, 1):
        X = rng.standard_normal((g.n, nv))
        Y0 = np.zeros((g.n, nv))
        na, al = both(g, X, Y0, "N", 1.0, 0.0)
        want = ref.gemv(X)
        B = ref.gemv(X, absval=True)
        assert np.all(np.abs(na - want) <= 1e-12 * B), (nv, np.max(np.abs(na - want) / B))
        assert np.all(np.abs(na - al) <= 2e-12 * B), nv
        if nv == 1:
            assert np.array_equal(na, al)
    g.close()
    ref.close()


@pytest.mark.parametrize("schedule", [0, 1, 2, 3])
def test_noalloc_under_every_schedule(schedule):
    """The no-allocation product follows the handle's schedule on its own
    side stream (schedule 3, which needs a third stream that the fixed
    scratch views do not have, runs as schedule 2): with passes of the same
    width as h2_gemv it gives h2_gemv's bits."""
    from paper_2109_05451_amd import H2Operator
    buf = np.array(h2gen.build_config("c1_2d_4096").array, copy=True)
    g = H2Operator(buf)
    g.set_schedule("fp64", schedule)
    rng = np.random.default_rng(30 + schedule)
    for nv in (1, 3):
        X = rng.standard_normal((g.n, nv))
        Y0 = rng.standard_normal((g.n, nv))
        na, al = both(g, X, Y0, "N", 1.0, 0.5)
        assert np.array_equal(na, al), (schedule, nv)
    g.close()
