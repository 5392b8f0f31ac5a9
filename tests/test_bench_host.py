"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the algorithmic
flop and byte counts, the whole-path roofline and the traffic lookup in the
committed profile summaries."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def stats(**kw):
    st = {"n": 1000, "tree_rows": 300, "entries_U": 0, "entries_V": 0, "entries_E": 0, "entries_F": 0,
          "entries_S": 0, "entries_D": 0}
    st.update(kw)
    return st


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_flop_count_convention():
    """2 nv flops per stored entry, plus n nv for alpha and 2 n nv when beta != 0."""
    st = stats(entries_U=10, entries_V=20, entries_E=3, entries_F=4, entries_S=100, entries_D=50)
    a = bench.algorithmic(st, 3)
    assert a["flops"] == 2 * 3 * 187 + 1000 * 3
    assert bench.algorithmic(st, 3, beta_nonzero=True)["flops"] == 2 * 3 * 187 + 3 * 1000 * 3
    assert a["phase_flops"]["coupling"] == 2 * 3 * 100 and a["phase_flops"]["dense"] == 2 * 3 * 50
    assert a["phase_bytes"]["coupling"] == 8 * 100 + 2 * 8 * 3 * 300


def test_path_roofline_bytes_and_flops():
    # nv = 1: 8 bytes and 2 flops per entry, far under every ridge: bound by HBM
    st = stats(entries_S=10 ** 9, entries_D=10 ** 9)
    r = bench.path_roofline(st, 1, "fp64", 10.0)
    t_bytes = (16e9 + 8.0 * 1000 * 2 + 4 * 8.0 * 300) / 8e12 * 1e3
    assert r["bound"] == "hbm" and abs(r["t_roof_ms"] - round(t_bytes, 4)) < 1e-4
    assert abs(r["frac"] - round(r["t_roof_ms"] / 10.0, 4)) < 1e-4
    # nv = 64 in BF16: the low-rank bytes shrink 4x, the FP64 dense flops set the bound
    r16 = bench.path_roofline(st, 64, "bf16", 10.0)
    t_flops = 2 * 64 * 1e9 / 2500e12 + 2 * 64 * 1e9 / 78.6e12
    assert r16["bound"] == "flops" and abs(r16["t_roof_ms"] - round(t_flops * 1e3, 4)) < 1e-4


def test_traffic_only_from_a_summary_of_the_same_kernel_source(tmp_path, monkeypatch):
    src = tmp_path / "paper_2109_05451_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "h2_kernels.hip").write_bytes(b"// kernels\n")
    (src / "h2_tree_kernels.hip").write_bytes(b"// more kernels\n")
    md5 = hashlib.md5(b"// kernels\n// more kernels\n").hexdigest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k_rows_cfg_nv1.md").write_text(f"kernel_source_md5: `{md5}`\n\n"
                                            "traffic_bytes_per_launch (coupling rows): 1.5e+09\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("cfg", 1, "coupling") == 1.5e9
    assert bench.measured_traffic("cfg", 1, "dense") is None       # no figure for that launch
    assert bench.measured_traffic("cfg", 64, "coupling") is None   # no summary for that workload
    assert bench.measured_traffic("cfg", 1, "coupling", "bf16") is None  # no summary for that precision
    (src / "h2_tree_kernels.hip").write_bytes(b"// more kernels, changed\n")
    assert bench.measured_traffic("cfg", 1, "coupling") is None    # taken on another kernel source
    # a summary that names the priced kernel's own file: other files may change
    one = hashlib.md5(b"// kernels\n").hexdigest()
    (prof / "k_rows_cfg_nv16.md").write_text(f"kernel_source_md5: `{one}` (of: h2_kernels.hip)\n\n"
                                             "traffic_bytes_per_launch (coupling rows): 2.5e+09\n")
    assert bench.measured_traffic("cfg", 16, "coupling") == 2.5e9
    (src / "h2_kernels.hip").write_bytes(b"// kernels, changed\n")
    assert bench.measured_traffic("cfg", 16, "coupling") is None


def test_plan_description_parsing():
    """The tuned coupling time and the launch count read from h2_plan_info's
    text: the schedule decides which coupling lines count; launches marked
    skipped do not count."""
    info = "\n".join([
        "first level with coupling blocks: 3 (sweep transfers above it skipped)",
        "fp64: coupling rows longest first, dense rows longest first",
        "fp64: dense schedule 0 (tuned products 3.0 / 3.1 / 3.1 / 3.2 ms)",
        "fp32: dense schedule 3 (tuned products 2.7 / 2.7 / 2.7 / 2.6 ms)",
        "up rows=4 max_rows=36 kind=0 | fp64 kc=9 grid=0 xcd=0 fl=0 occ=0 0.010ms | skipped (above the first "
        "coupling level)",
        "up rows=8 max_rows=36 kind=0 | fp64 kc=9 grid=0 xcd=0 fl=0 occ=0 0.012ms",
        "couple rows=100 max_rows=36 kind=0 | fp64 kc=9 grid=0 xcd=0 fl=1 occ=5 1.127ms | fp32 kc=9 grid=0 xcd=0 "
        "fl=1 occ=0 0.950ms",
        "couple_deep rows=60 max_rows=36 kind=0 | fp64 kc=9 grid=0 xcd=0 fl=1 occ=0 0.700ms | fp32 kc=9 grid=0 "
        "xcd=0 fl=1 occ=0 0.600ms",
        "couple_rest rows=40 max_rows=36 kind=0 | fp64 kc=9 grid=0 xcd=0 fl=1 occ=5 0.400ms | fp32 kc=9 grid=0 "
        "xcd=0 fl=0 occ=0 0.300ms",
        "down rows=8 max_rows=36 kind=0 | fp64 kc=9 grid=0 xcd=0 fl=0 occ=0 0.011ms",
        "dense1 rows=50 max_rows=64 kind=0 | fp64 kc=9 grid=0 xcd=0 fl=0 occ=0 0.500ms",
        "out rows=50 max_rows=64 kind=0 | fp64 kc=9 grid=0 xcd=0 fl=0 occ=0 0.080ms",
    ])
    assert abs(bench.tuned_coupling_ms(info, "fp64") - 1.127) < 1e-9       # schedule 0: the one launch
    assert abs(bench.tuned_coupling_ms(info, "fp32") - 0.9) < 1e-9         # schedule 3: deep + rest

    class G:
        def plan_info(self):
            return info
    # permutation + up (one of two runs) + couple + down + dense1 + out
    assert bench.launches_per_product(G()) == 1 + 1 + 1 + 1 + 1 + 1
