"""The FP64 oracle built with g++ and the address and undefined-behaviour
sanitizers, run over every exported function on small lattices of each theory
(oracle/sanitize_check.cpp). Host code only; no GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_is_clean_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", *san, "-o", exe,
                           os.path.join(ROOT, "oracle", "oracle.cpp"),
                           os.path.join(ROOT, "oracle", "sanitize_check.cpp")])
    # a library preloaded by the environment may come before the sanitizer runtime
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok"
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
