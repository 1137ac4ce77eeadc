"""The host plan builder (plan.cpp) under AddressSanitizer and
UndefinedBehaviorSanitizer: tests/host_plan_fuzz.cpp builds the workload
plans, edge cases and 400 seeded random parameter sets and checks the
invariants the kernels index with. g++ only: no device code is built."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2603_29785_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_plan_builder_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_plan_fuzz")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           os.path.join(HERE, "host_plan_fuzz.cpp"), os.path.join(CSRC, "plan.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "0 failures" in r.stdout
