"""Compile the C oracle into oracle/libspamm_oracle.so (host code, gcc, OpenMP).

Portable x86-64 code generation (no -march=native) so the library built here also
runs on other hosts.  FP contraction is off so each multiply and add rounds on its
own, as written in the C source.
"""

from __future__ import annotations

import subprocess
from pathlib import Path

HERE = Path(__file__).resolve().parent
SRC = HERE / "spamm_oracle.c"
OUT = HERE / "libspamm_oracle.so"


def build_oracle(verbose: bool = False) -> Path:
    tmp = OUT.with_suffix(".so.tmp")
    cmd = [
        "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
        "-Wall", "-Wextra", "-o", str(tmp), str(SRC), "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    tmp.replace(OUT)
    return OUT


if __name__ == "__main__":
    print(build_oracle(verbose=True))
