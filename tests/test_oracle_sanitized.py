"""The oracle's pins under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): the C oracle is rebuilt with both, preloaded into a child
interpreter, and its pin tests must pass with no sanitizer report (any
report aborts the child: recovery is off)."""
import os
import subprocess
import sys

import pytest

from oracle import build as obuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_pins_under_asan_ubsan():
    try:
        lib = obuild.build(sanitize=True)
        rt = obuild.asan_runtime()
    except (OSError, subprocess.CalledProcessError) as e:
        pytest.skip(f"sanitizer build unavailable: {e}")
    if not os.path.isabs(rt):
        pytest.skip("gcc has no AddressSanitizer runtime")
    env = dict(os.environ, LD_PRELOAD=rt, PLUQ_ORACLE_LIB=lib, OMP_NUM_THREADS="4",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
           os.path.join(ROOT, "tests", "test_oracle.py"), os.path.join(ROOT, "tests", "test_oracle_post.py")]
    res = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert " passed" in out
