"""The oracle's pin tests once more, with the oracle built under
AddressSanitizer and UndefinedBehaviorSanitizer (gcc -fsanitize=address,undefined,
no recovery): an out-of-bounds access, a use after free or undefined behaviour
anywhere in the C oracle on those inputs aborts the run.  The pins run in a
child Python process that preloads the sanitizer runtime (Python itself is not
instrumented; its own allocations are not leak-checked)."""

from __future__ import annotations

import os
import subprocess
import sys
from pathlib import Path

import pytest

from oracle import build as ob

ROOT = Path(__file__).resolve().parent.parent


@pytest.mark.slow
def test_oracle_pins_under_asan_and_ubsan():
    lib = ob.build_oracle(sanitize=True)
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": ob.sanitizer_runtime(),
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
        "SPAMM_ORACLE_LIB": str(lib),
        "OMP_NUM_THREADS": "4",
    })
    probe = subprocess.run([sys.executable, "-c", "import ctypes, oracle; oracle._load(); "
                            "print(oracle.LIB_PATH, hasattr(ctypes.CDLL(None), '__asan_init'))"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert probe.stdout.split() == [str(lib), "True"], probe.stdout + probe.stderr  # the sanitized build, ASan live
    pins = ["tests/test_oracle_pins.py", "tests/test_learned_oracle.py"]
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider", *pins],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert " passed" in out
