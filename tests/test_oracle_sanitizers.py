"""The CPU oracle built with the address and undefined-behaviour sanitizers
(gcc, host code only) traces rays of every model (thermal IQUV and I with
subrings, toy disk, a small gridded snapshot, a screen function) on two
threads without a sanitizer report and with finite results."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-D_GNU_SOURCE", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-o", exe, os.path.join(ORACLE, "sanitize_main.c"), "-lm", "-lpthread"]
    subprocess.check_call(cmd, cwd=ORACLE)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], cwd=ORACLE, env=env, capture_output=True, text=True, timeout=600)
    print(r.stdout)
    print(r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert r.stdout.strip().endswith("OK")
