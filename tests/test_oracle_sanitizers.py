"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only) and driven through every entry point by
oracle/sanitize_driver.c: no out-of-bounds access, leak, or undefined
operation, and the photon ledgers of the small problems close.  No GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    exe = tmp_path / "oracle_sanitized"
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "oracle"), "-o", str(exe),
           os.path.join(ROOT, "oracle", "sanitize_driver.c"), os.path.join(ROOT, "oracle", "traphic_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "sanitize driver OK" in r.stdout
    assert "runtime error" not in r.stderr
