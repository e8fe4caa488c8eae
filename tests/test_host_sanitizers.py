"""The library's host planner under AddressSanitizer and UBSan (CPU only).

geometry.cpp (validation, cluster enumeration, contraction plans, partition
listing and coefficients) is plain host C++: it is built here with g++ and
the sanitizers, and driven through lattices, open legs, partitions,
sub-partitions and malformed descriptors (tests/host/geometry_driver.cpp).
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_planner_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = tmp_path / "geometry_driver"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2512_10910_amd", "csrc"),
           os.path.join(ROOT, "paper_2512_10910_amd", "csrc", "geometry.cpp"),
           os.path.join(ROOT, "tests", "host", "geometry_driver.cpp"), "-o", str(exe)]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "ok (0 failures)" in out.stdout
