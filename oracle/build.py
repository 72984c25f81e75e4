"""Compile the C oracle (host code, gcc, OpenMP).

Three variants of the same source, ``spamm_oracle.c``:

* ``libspamm_oracle.so`` — what the tests load: -O3 with portable x86-64
  code generation, so the library built on one host also runs on another.
* ``libspamm_oracle_native.so`` (``build_oracle(native=True)``) — -O3
  -march=native, built on the host that runs it, for timing the oracle as a
  CPU baseline.
* ``libspamm_oracle_san.so`` (``build_oracle(sanitize=True)``) — AddressSanitizer
  and UndefinedBehaviorSanitizer, for running the oracle's pin tests under
  both (the Python process preloads the sanitizer runtime).

FP contraction is off in every variant so each multiply and add rounds on its
own, as written in the C source, and no variant may reassociate FP arithmetic
(no -ffast-math): the three compute the same bits.
"""

from __future__ import annotations

import subprocess
from pathlib import Path

HERE = Path(__file__).resolve().parent
SRC = HERE / "spamm_oracle.c"
OUT = HERE / "libspamm_oracle.so"
OUT_NATIVE = HERE / "libspamm_oracle_native.so"
OUT_SAN = HERE / "libspamm_oracle_san.so"

BASE = ["-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-Wall", "-Wextra"]
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def output_path(*, native: bool = False, sanitize: bool = False) -> Path:
    return OUT_SAN if sanitize else OUT_NATIVE if native else OUT


def build_oracle(verbose: bool = False, *, native: bool = False, sanitize: bool = False) -> Path:
    out = output_path(native=native, sanitize=sanitize)
    opt = SAN if sanitize else ["-O3", "-march=native"] if native else ["-O3"]
    tmp = out.with_suffix(".so.tmp")
    cmd = ["gcc", *opt, *BASE, "-o", str(tmp), str(SRC), "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    tmp.replace(out)
    return out


def sanitizer_runtime() -> str:
    """Path of gcc's AddressSanitizer runtime (to preload into Python)."""
    return subprocess.run(["gcc", "-print-file-name=libasan.so"], check=True, capture_output=True,
                          text=True).stdout.strip()


if __name__ == "__main__":
    print(build_oracle(verbose=True))
