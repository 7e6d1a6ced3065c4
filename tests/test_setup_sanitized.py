"""The library's host set-up code (csrc/setup.cpp) under AddressSanitizer and
UndefinedBehaviorSanitizer: tests/host/setup_sanitize.cpp drives assembly,
elimination, lifting of prescribed values, the multigrid hierarchy, batch
concatenation, the folded operators and the argument checks on 2D and 3D
meshes; the build is plain g++ (host code only), and any sanitizer report or
failed check fails the test."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_setup_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "setup_sanitize")
    src = [os.path.join(HERE, "host", "setup_sanitize.cpp"),
           os.path.join(ROOT, "paper_2310_10430_amd", "csrc", "setup.cpp")]
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", *src, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout
