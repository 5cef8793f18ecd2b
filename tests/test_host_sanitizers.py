"""The C code of the oracle and of the input generators, built with
AddressSanitizer and UndefinedBehaviorSanitizer (gcc, host only; every report
aborts) and run through degenerate cases by tests/host/sanitize_driver.c."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_and_generators_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "sanitize_driver")
    srcs = [os.path.join(ROOT, "tests", "host", "sanitize_driver.c"), os.path.join(ROOT, "oracle", "uf_oracle.c"),
            os.path.join(ROOT, "synth", "streamgen.c")]
    flags = ["-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all"]
    subprocess.check_call(["gcc"] + flags + ["-o", exe] + srcs + ["-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sanitized host checks passed" in r.stdout
