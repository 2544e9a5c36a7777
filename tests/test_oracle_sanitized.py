"""The oracle built with the address and undefined-behaviour sanitizers
(g++, host code only) runs a small three-level run with regrids, a refine point
and a fixed-grid run through its C interface without a report
(`tests/sanitize_driver.cpp`)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_oracle_under_sanitizers():
    ora = os.path.join(ROOT, "oracle")
    srcs = [os.path.join(ROOT, "tests", "sanitize_driver.cpp")] + \
        [os.path.join(ora, f) for f in ("ora_amr.cpp", "ora_adjoint.cpp", "ora_count.cpp")]
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "san")
        subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
                               "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                               "-ffp-contract=off", "-I" + ora] + srcs + ["-o", exe])
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    assert r.stdout.strip().endswith("ok")
