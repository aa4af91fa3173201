"""The oracle's C++ under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only): every entry point runs on small seeded inputs of one to four
words per key, and any invalid access, leak or undefined operation fails."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_sanitized"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
                           "-ffp-contract=off", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all",
                           os.path.join(ROOT, "oracle", "iqcc_oracle.cpp"),
                           os.path.join(HERE, "oracle_sanitize_driver.cpp"), "-o", str(exe)])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok"), r.stdout + r.stderr
