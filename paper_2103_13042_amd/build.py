"""Build libspamm.so for gfx950 with hipcc (in-tree, next to this file).

    python -m paper_2103_13042_amd.build

Flags: gfx950 code only; packed-FP32 instructions disabled; FP32 denormals kept
(inputs of decay matrices reach the FP32 subnormal range and their squares
must enter the FP64 norm sums unchanged).
"""

from __future__ import annotations

import os
import subprocess
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
INCLUDE = ROOT / "include"
LIB = PKG / "libspamm.so"
SOURCES = [CSRC / "kernels.hip", CSRC / "multiply_macro.hip", CSRC / "multiply_lowp.hip", CSRC / "multiply_small.hip",
           CSRC / "split.hip", CSRC / "learned.hip", CSRC / "api.hip", CSRC / "api_tau.hip", CSRC / "api_batch.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cand = Path(rocm) / "bin" / "hipcc"
    return str(cand) if cand.exists() else "hipcc"


def compile_flags() -> list[str]:
    return [
        f"--offload-arch={ARCH}",
        "-O3",
        "-std=c++17",
        "-fPIC",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-fno-gpu-flush-denormals-to-zero",
        "-Wall",
        f"-I{INCLUDE}",
        f"-I{CSRC}",
    ]


def build_library(verbose: bool = False, jobs: int = 3) -> Path:
    """Compile every HIP source of the library and link libspamm.so."""
    objs = []
    procs = []
    env = dict(os.environ)
    for src in SOURCES:
        obj = PKG / "_build" / (src.stem + ".o")
        obj.parent.mkdir(exist_ok=True)
        cmd = [hipcc(), *compile_flags(), "-c", str(src), "-o", str(obj)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, env=env), cmd))
        objs.append(obj)
        if len(procs) >= jobs:
            p, c = procs.pop(0)
            if p.wait() != 0:
                raise RuntimeError("hipcc failed: " + " ".join(c))
    for p, c in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed: " + " ".join(c))
    tmp = LIB.with_suffix(".so.tmp")
    link = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", str(tmp), *map(str, objs)]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True, env=env)
    tmp.replace(LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
