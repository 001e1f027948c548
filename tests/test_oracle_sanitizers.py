"""The CPU oracle under the host address and undefined-behaviour sanitizers.

tests/oracle_sanitize_driver.c calls the oracle's entry points on small inputs
(a zero-variance stock, labels out of range, N = 1, both selections with the
termination test, both EWMA modes, brute force over Bell(6) partitions); built
with gcc -fsanitize=address,undefined and run as a child process, it must exit
0 with no sanitizer report. Skipped when gcc or the sanitizer runtimes are
missing."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_runs_clean_under_asan_and_ubsan():
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "drv")
        cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=all", os.path.join(HERE, "oracle_sanitize_driver.c"),
               os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", exe]
        b = subprocess.run(cmd, capture_output=True, text=True)
        if b.returncode != 0:
            pytest.skip("sanitizer build unavailable: " + b.stderr[-300:])
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
        assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
        assert r.stdout.startswith("ok")
