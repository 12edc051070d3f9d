"""The oracle's C code built with AddressSanitizer and UndefinedBehaviorSanitizer and
driven through every entry point on small inputs (host code only; no GPU)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_address_and_ub_sanitizers():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "oracle_san")
        cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-fno-omit-frame-pointer", "-pthread", os.path.join(ROOT, "oracle", "grtx_oracle.c"),
               os.path.join(ROOT, "tests", "csan", "oracle_driver.c"), "-lm", "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0 and "sanitize" in r.stderr and "unrecognized" in r.stderr:
            pytest.skip("this gcc has no sanitizer runtime")
        assert r.returncode == 0, r.stderr[-2000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
        run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
        assert run.returncode == 0, (run.stdout[-1000:], run.stderr[-3000:])
        assert run.stdout.startswith("ok")
