"""Build libspamm.so for gfx950 with hipcc (in-tree, next to this file).

    python -m paper_2103_13042_amd.build

Each source is compiled in two passes: the device pass (gfx950 code only,
packed-FP32 instructions disabled, FP32 denormals kept: inputs of decay
matrices reach the FP32 subnormal range and their squares must enter the FP64
norm sums unchanged) writes the offload bundle, and the host pass embeds it.
The packed-FP32 feature only exists for the device target, so the host pass
does not get it.  ``packed_fp32_instructions`` disassembles the gfx950 code
built here and lists any packed FP32 instruction left in it.
"""

from __future__ import annotations

import os
import re
import subprocess
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
INCLUDE = ROOT / "include"
LIB = PKG / "libspamm.so"
BUILD = PKG / "_build"
SOURCES = sorted(CSRC.glob("*.hip"))  # every kernel and entry-point source of the library
ARCH = "gfx950"
TARGET = f"hipv4-amdgcn-amd-amdhsa--{ARCH}"


def rocm() -> Path:
    return Path(os.environ.get("ROCM_PATH", "/opt/rocm"))


def hipcc() -> str:
    cand = rocm() / "bin" / "hipcc"
    return str(cand) if cand.exists() else "hipcc"


def common_flags() -> list[str]:
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", f"-I{INCLUDE}", f"-I{CSRC}"]


def device_flags() -> list[str]:
    return ["--offload-device-only", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-fno-gpu-flush-denormals-to-zero"]


def compile_commands(src: Path) -> tuple[list[str], list[str], Path]:
    """(device pass, host pass, object) for one source."""
    bundle = BUILD / (src.stem + ".hipfb")
    obj = BUILD / (src.stem + ".o")
    dev = [hipcc(), *common_flags(), *device_flags(), "-c", str(src), "-o", str(bundle)]
    host = [hipcc(), *common_flags(), "--offload-host-only", "-Xclang", "-fcuda-include-gpubinary", "-Xclang",
            str(bundle), "-c", str(src), "-o", str(obj)]
    return dev, host, obj


def build_library(verbose: bool = False, jobs: int = 3) -> Path:
    """Compile every HIP source of the library and link libspamm.so."""
    BUILD.mkdir(exist_ok=True)
    env = dict(os.environ)
    objs, running = [], []

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        return subprocess.Popen(cmd, env=env)

    def finish(entry):
        proc, cmd, host = entry
        if proc.wait() != 0:
            raise RuntimeError("hipcc failed: " + " ".join(cmd))
        if host is not None:  # the host pass needs the bundle of the device pass
            p2 = run(host)
            if p2.wait() != 0:
                raise RuntimeError("hipcc failed: " + " ".join(host))

    for src in SOURCES:
        dev, host, obj = compile_commands(src)
        running.append((run(dev), dev, host))
        objs.append(obj)
        if len(running) >= jobs:
            finish(running.pop(0))
    for entry in running:
        finish(entry)
    tmp = LIB.with_suffix(".so.tmp")
    link = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", str(tmp), *map(str, objs)]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True, env=env)
    tmp.replace(LIB)
    return LIB


_PACKED_FP32 = re.compile(r"\bv_pk_(fma|mul|add)_f32\b")


def packed_fp32_instructions() -> list[str]:
    """Packed FP32 instructions in the gfx950 code objects of the last build
    (each bundle unbundled and disassembled); empty when there are none."""
    llvm = rocm() / "lib" / "llvm" / "bin"
    found = []
    for bundle in sorted(BUILD.glob("*.hipfb")):
        co = bundle.with_suffix(".co")
        subprocess.run([str(llvm / "clang-offload-bundler"), "--type=o", f"--targets={TARGET}",
                        f"--input={bundle}", f"--output={co}", "--unbundle"], check=True)
        asm = subprocess.run([str(llvm / "llvm-objdump"), "-d", f"--mcpu={ARCH}", str(co)], check=True,
                             capture_output=True, text=True).stdout
        found += [f"{bundle.stem}: {line.strip()}" for line in asm.splitlines() if _PACKED_FP32.search(line)]
        co.unlink()
    return found


if __name__ == "__main__":
    print(build_library(verbose=True))
