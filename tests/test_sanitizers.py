"""The host planner (index sets, plans, block sets, factor trees and their
parse, multiplicities, tensor e-graphs) built with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer and run on every operator family (no GPU).

Only host C++ is instrumented: the HIP kernels are not compiled here.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2201_04269_amd", "csrc")
SOURCES = ["index_set.cpp", "block_set.cpp", "plan.cpp", "egraph.cpp", "factor_tree.cpp"]


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_planner_is_clean_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "sanitize_host"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, os.path.join(ROOT, "tests", "sanitize_host.cpp")]
    cmd += [os.path.join(CSRC, s) for s in SOURCES] + ["-o", str(exe)]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=900)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "sanitized host run ok" in r.stdout
