"""The pins are sensitive: plausible mistakes planted in a copy of the oracle
(on the CPU) must each be caught by at least one pin.

Each mutant is a textual edit of ``oracle/h2_oracle.c`` -- a transposed
operand, a dropped term, a wrong sign or index, swapped bases -- compiled to a
temporary library and swapped in for the real one while a compact set of pins
runs.
"""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

import h2gen
import oracle
from tests.brute import dense_original_order

SRC = os.path.join(os.path.dirname(oracle.__file__), "h2_oracle.c")

MUTANTS = {
    "transfer_transposed": ("A(Tc[a + k[l] * b], absval)", "A(Tc[b + k[l - 1] * a], absval)"),
    "coupling_transposed": ("Sg[b + r->krow[l] * a] : Sg[a + r->krow[l] * b]",
                            "Sg[b + r->krow[l] * a] : Sg[b + r->krow[l] * a]"),
    "beta_sign": ("*y = al * Z[i + n * v] + (beta", "*y = al * Z[i + n * v] - (beta"),
    "leaf_sum_off_by_one": ("j < r->leafend[s]; ++j", "j < r->leafend[s] - 1; ++j"),
    "root_level_dropped": ("for (int64_t l = q; l >= 0; --l) {\n        const int64_t k = w.krow[l];",
                           "for (int64_t l = q; l >= 1; --l) {\n        const int64_t k = w.krow[l];"),
    "input_not_permuted": ("xt[i + n * v] = X[r->perm[i] + ldx * v];\n    rc = core",
                           "xt[i + n * v] = X[i + ldx * v];\n    rc = core"),
    "column_basis_is_row_basis": ("w.Bcol = r->V; w.Tcol = r->F;", "w.Bcol = r->U; w.Tcol = r->F;"),
    "dense_transposed_read": ("double d = trans ? Db[jj + mt * i] : Db[i + mt * jj];",
                              "double d = trans ? Db[jj + mt * i] : Db[jj + mt * i];"),
    "dense_dropped": ("s += A(d, absval) * A(xt[r->lo[other] + jj + r->n * v], absval);",
                      "s += 0.0 * A(d, absval);"),
    "transpose_uses_rows": ("bbeg = r->sc_ptr[t];\n      bend = r->sc_ptr[t + 1];",
                            "bbeg = r->sc_ptr[t];\n      bend = r->sc_ptr[t];"),
}


def _pins_pass():
    """Compact pin set: integer brute force (both ops, alpha/beta) on a few
    tiny trees, and the exact polynomial-kernel closed form."""
    try:
        for seed, kw in [(1, dict(q=2)), (2, dict(q=3, separate=True)), (3, dict(q=3, max_children=2)),
                         (4, dict(q=1))]:
            buf = h2gen.random_rep(seed, **kw)
            A = dense_original_order(buf)
            o = oracle.Oracle(buf)
            rng = np.random.default_rng(seed)
            X = rng.integers(-2, 3, size=(o.n, 2)).astype(float)
            Y0 = rng.integers(-2, 3, size=(o.n, 2)).astype(float)
            for op, M in (("N", A), ("T", A.T)):
                if not np.array_equal(o.gemv(X, op=op, alpha=2.0, beta=-1.0, Y=Y0), 2.0 * M @ X - Y0):
                    return False
        P = h2gen.points(800, 2, 21)
        buf = h2gen.build(P, leaf=32, p=3, eta=0.9, kernel="poly2")
        X = h2gen.vectors(800, 1, 1)
        want = (1.0 + P @ P.T) ** 2 @ X
        got = oracle.Oracle(buf.array).gemv(X)
        return np.linalg.norm(got - want) <= 1e-11 * np.linalg.norm(want)
    except oracle.OracleError:
        return False


def test_unmutated_oracle_passes_compact_pins():
    assert _pins_pass()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique/present"
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "m.c")
        so = os.path.join(d, "m.so")
        open(c, "w").write(src.replace(old, new))
        subprocess.run(["gcc", "-O1", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o", so, c, "-lm"],
                       check=True)
        real = oracle._load()
        mut = ctypes.CDLL(so)
        for fn in ("h2o_open", "h2o_close", "h2o_n", "h2o_gemv", "h2o_gemv_rows", "h2o_dense"):
            f = getattr(mut, fn)
            f.argtypes = getattr(real, fn).argtypes
            f.restype = getattr(real, fn).restype
        monkeypatch.setattr(oracle, "_lib", mut)
        assert not _pins_pass(), f"planted mistake '{name}' passed every pin"
