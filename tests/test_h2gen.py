"""The input generator: buffer lifetime and the structure of built operators
(the leaf blocks partition I x J, perm is a permutation, child ranges tile
their parent, every leaf on level q with size at most the leaf size)."""
import gc

import numpy as np
import pytest

import h2gen
import oracle
from h2gen import fmt


def test_view_outlives_builder_object():
    a = h2gen.build(h2gen.points(3000, 3, 3), leaf=64, p=3, eta=0.7, kernel="laplace").array
    gc.collect()
    junk = np.ones(20_000_000)  # reuse freed memory if the view were dangling
    del junk
    assert oracle.try_open(a) == 0
    b = h2gen.build_config("c1_2d_4096")
    view = b.array
    b.free()
    del b
    gc.collect()
    assert oracle.try_open(view) == 0


@pytest.mark.parametrize("n,dim,leaf,eta", [(1000, 2, 32, 0.7), (3000, 3, 48, 0.7), (777, 2, 20, 1.5),
                                            (4096, 2, 64, 0.0)])
def test_blocks_partition_the_matrix(n, dim, leaf, eta):
    r = fmt.parse(h2gen.build(h2gen.points(n, dim, 1), leaf=leaf, p=3, eta=eta, kernel="exp").array)
    q, lp, lo, hi = r["q"], r["level_ptr"], r["lo"], r["hi"]
    cover = np.zeros((n, n), dtype=np.int32)
    for l in range(q + 1):
        rp, cl = r["s_rowptr"][l], r["s_col"][l]
        for ti in range(int(lp[l + 1] - lp[l])):
            t = int(lp[l]) + ti
            for b in range(int(rp[ti]), int(rp[ti + 1])):
                s = int(lp[l]) + int(cl[b])
                assert t != s
                cover[lo[t]:hi[t], lo[s]:hi[s]] += 1
    leaf0 = int(lp[q])
    for ti in range(int(lp[q + 1] - lp[q])):
        for b in range(int(r["d_rowptr"][ti]), int(r["d_rowptr"][ti + 1])):
            t, s = leaf0 + ti, leaf0 + int(r["d_col"][b])
            cover[lo[t]:hi[t], lo[s]:hi[s]] += 1
    assert np.all(cover == 1)
    assert np.array_equal(np.sort(r["perm"]), np.arange(n))
    sizes = hi[leaf0:] - lo[leaf0:]
    assert sizes.max() <= leaf and sizes.min() >= 1
    for c in range(1, r["nnodes"]):
        p = r["parent"][c]
        assert lo[p] <= lo[c] <= hi[c] <= hi[p]
