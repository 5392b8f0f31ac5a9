"""Checks on the gfx950 assembly of the library's kernels (CPU only: hipcc
cross-compiles).

An MFMA's result may be read only after the wait states its pipeline needs;
the compiler inserts them as s_nop before the first read.  One kernel form
(an 8-column vector-tile kernel, since taken out) compiled to an epilogue
that read one accumulator register and only then waited, and gave wrong
bits on the GPU.  This test compiles every kernel source as the build does
and fails if any accumulator read is directly followed by a long s_nop,
the mark of that misplaced wait."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2109_05451_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def late_waits(asm_text):
    """(function, read, nop) for each accumulator read followed at once by
    an s_nop of 4 or more wait states."""
    out, fn, prev = [], None, None
    for line in asm_text.splitlines():
        m = re.match(r"^(_Z\S+):", line)
        if m:
            fn, prev = m.group(1), None
            continue
        s = line.strip()
        if not s or s.startswith((";", ".")):
            continue
        if s.startswith("s_nop") and prev and prev.startswith("v_accvgpr_read"):
            if int(s.split()[1]) >= 4:
                out.append((fn, prev, s))
        prev = s
    return out


def test_scanner_finds_the_pattern():
    bad = "_Zk:\n\tv_mfma_f64_16x16x4_f64 a[0:7], v[0:1], v[2:3], a[0:7]\n\tv_accvgpr_read_b32 v9, a7\n\ts_nop 10\n"
    good = "_Zk:\n\tv_mfma_f64_16x16x4_f64 a[0:7], v[0:1], v[2:3], a[0:7]\n\ts_nop 11\n\tv_accvgpr_read_b32 v9, a7\n"
    assert len(late_waits(bad)) == 1
    assert late_waits(good) == []


@pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which(HIPCC)), reason="hipcc not available")
@pytest.mark.parametrize("src", ["h2_kernels.hip", "h2_compress_kernels.hip"])
def test_no_accumulator_read_before_its_wait(src, tmp_path):
    out = tmp_path / (src + ".s")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-I" + os.path.join(ROOT, "include"), "--cuda-device-only", "-S",
                    os.path.join(CSRC, src), "-o", str(out)],
                   check=True, cwd=tmp_path, capture_output=True)
    hits = late_waits(out.read_text())
    assert hits == [], hits[:3]
