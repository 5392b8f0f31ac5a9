"""C-ABI library checks that need no GPU: every symbol declared in
include/h2.h is exported, and the host-side validator agrees with the
oracle's independent reader on valid and corrupted representations."""
import os
import re

import numpy as np
import pytest

import h2gen
import oracle
import paper_2109_05451_amd as lib
from h2gen import fmt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "h2.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(h2_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("h2_load", "h2_load_mem", "h2_gemv", "h2_free", "h2_last_error", "h2_stats"):
        assert required in names
    assert set(names) == set(lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    so = lib.load_library()
    for name in declared_functions():
        assert hasattr(so, name), name


def test_validate_accepts_builder_and_random_reps():
    assert lib.validate(h2gen.build_config("c1_2d_4096").array) == lib.H2_OK
    for seed in range(10):
        assert lib.validate(h2gen.random_rep(seed, q=3, allow_empty=True)) == lib.H2_OK


@pytest.mark.parametrize("mutate", ["magic", "version", "truncate", "perm", "dense_col", "tree_lo",
                                    "tree_parent", "csr_order", "flags", "total"])
def test_validate_rejects_like_the_oracle(mutate):
    buf = np.array(h2gen.random_rep(1, q=3, p_adm=0.2), copy=True)
    r = fmt.parse(buf)
    if mutate == "magic":
        buf[1] = ord("Z")
    elif mutate == "version":
        buf[8] = 7
    elif mutate == "truncate":
        buf = buf[:-64]
    elif mutate == "perm":
        r["perm"][-1] = r["perm"][0]
    elif mutate == "dense_col":
        r["d_col"][0] = -1
    elif mutate == "tree_lo":
        r["hi"][1] -= 1
    elif mutate == "tree_parent":
        r["parent"][int(r["level_ptr"][2])] = 0  # level-2 node pointing at the root
    elif mutate == "csr_order":
        c = r["d_col"]
        rp = r["d_rowptr"]
        row = int(np.argmax(np.diff(rp) >= 2))
        assert rp[row + 1] - rp[row] >= 2
        b = int(rp[row])
        c[b], c[b + 1] = c[b + 1], c[b]
    elif mutate == "flags":
        buf[13] = 1
    elif mutate == "total":
        buf[96] += 64
    rc = lib.validate(buf)
    assert rc in (lib.H2_EFORMAT, lib.H2_EINVAL), rc
    assert oracle.try_open(buf) != 0


def test_validate_rejects_unsupported_leaf():
    P = h2gen.points(600, 2, 1)
    buf = h2gen.build(P, leaf=300, p=2, eta=0.7, kernel="exp")
    assert fmt.parse(buf.array)["q"] == 1
    assert lib.validate(buf.array) == lib.H2_EUNSUPPORTED
