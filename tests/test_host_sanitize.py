"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the
representation reader and the launch-plan builder (h2_parse.cpp,
h2_plan.cpp) compiled with g++ together with tests/sanitize/host_check.cpp,
which parses builder output and seeded random representations, checks that
every planned row stays inside the section, vector tree or point array it
uses, and then parses seeded corruptions of each file from allocations of
exactly their length (see the harness's header).  A sanitizer report or a
bounds violation fails the test."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import h2gen
from h2gen import randrep

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2109_05451_amd", "csrc")


def _compile(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    exe = str(tmp_path / "host_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           os.path.join(ROOT, "tests", "sanitize", "host_check.cpp"),
           os.path.join(CSRC, "h2_parse.cpp"), os.path.join(CSRC, "h2_plan.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("sanitized host build unavailable: " + r.stderr[-400:])
    return exe


def test_reader_and_plan_under_sanitizers(tmp_path):
    exe = _compile(tmp_path)
    files = []
    reps = [h2gen.build(h2gen.points(900, 2, 11), 16, 3, 0.7, "exp", 0.1).array,
            h2gen.build(h2gen.points(700, 3, 12), 16, 2, 0.7, "laplace", 0.0).array]
    reps += [randrep.random_rep(s, q=3, p_adm=0.3) for s in range(4)]
    reps += [randrep.random_rep(10 + s, q=2, separate=False, allow_empty=False) for s in range(2)]
    for i, a in enumerate(reps):
        path = str(tmp_path / f"rep{i}.bin")
        np.asarray(a, dtype=np.uint8).tofile(path)
        files.append(path)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, "1500"] + files, capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-3000:]
    assert "FAIL" not in out and "runtime error" not in out and "AddressSanitizer" not in out, out[-3000:]
    lines = [ln for ln in r.stdout.splitlines() if " ok " in ln]
    assert len(lines) == len(files), out
    # the corruptions reach both outcomes: some are accepted (and planned), most rejected
    acc = sum(int(ln.split()[2]) for ln in lines)
    rej = sum(int(ln.split()[3]) for ln in lines)
    assert acc > 0 and rej > 0
