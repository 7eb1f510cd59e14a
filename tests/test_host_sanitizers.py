"""The host-side preparation and fusion code (csrc/ht_prep.cpp,
csrc/ht_fuse.cpp) built with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer and driven with random op sequences
(tests/host/sanitize_driver.cpp).  Host code only: no GPU, no HIP."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2604_15765_amd", "csrc")


def test_prep_and_fusion_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "sanitize_driver"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           f"-I{CSRC}", f"-I{os.path.join(ROOT, 'include')}",
           os.path.join(HERE, "host", "sanitize_driver.cpp"),
           os.path.join(CSRC, "ht_prep.cpp"), os.path.join(CSRC, "ht_fuse.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "failures 0" in r.stdout
