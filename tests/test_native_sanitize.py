"""The library's CPU-side code (generator, CSR transpose, red-black
preconditioner tables, small dense routines, tolerance controller) built with
g++ under AddressSanitizer and UndefinedBehaviorSanitizer and run on the
shapes the library meets: no sanitizer report, every check passes."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_code_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "sanitized")
    src = [os.path.join(ROOT, "tests", "native", "sanitize_main.cpp"),
           os.path.join(ROOT, "paper_2312_02891_amd", "csrc", "gen.cpp")]
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-o", exe] + src
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(p.stdout, p.stderr)
    assert p.returncode == 0, p.stderr
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr
    assert "0 failures" in p.stdout
