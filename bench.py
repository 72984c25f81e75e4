#!/usr/bin/env python3
"""Benchmark of the SpAMM hot path on one MI355X.

Default workload: algebraic-decay matrices A_ij = s_ij / (1 + |i-j|)^2 with
random signs (A seed 0, B seed 1), N = 8192, FP32, leaf tiles of 64, tau = 1e-6.

One step = one pass of the whole hot path over the resident inputs:
spamm_prepare_schedule (leaf norms of A and B, then the plan for tau and the
multiply schedule from one launch), then spamm_execute_scheduled (the MFMA
multiply kernel of the kept pairs).  (Reduced precision: the same first stage,
with the FP16 hi+lo scale exponents, spamm_prepare_schedule_scales, then the
in-register multiply; with the split planes spamm_prepare_split,
spamm_schedule, the planes' multiply.)  HIP events on the stream
the library launches on bracket K steps run back to back (the step time),
then K more steps with an event around each stage (the stage times; the
roofline figure uses the multiply launch's own time from these).  The other
thresholds of the sweep are timed before the headline threshold's warm-up.

  --write-traffic FETCH_CSV WRITE_CSV  turns two rocprofv3 --pmc runs of this
  script into profiles/multiply_traffic.json (HBM bytes per multiply launch).

Prints ONE JSON line on stdout; progress goes to stderr.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent
PEAK_FP32_MFMA_TFLOPS = 157.3  # MI355X dense FP32 matrix peak
PEAK_F16_MFMA_TFLOPS = 2500.0  # MI355X dense FP16 / BF16 matrix peak
METRIC = "dense-equiv TFLOP/s & speedup vs dense GEMM at rel. Frobenius err ≤1e-4"
TRAFFIC_FILE = ROOT / "profiles" / "multiply_traffic.json"
CSRC = ROOT / "paper_2103_13042_amd" / "csrc"
CALIB_BYTES = 256 << 20  # device copy whose counter readings scale the HBM byte counters


# the library's choice between the two forms of reduced-precision products:
# split planes from this many kept pairs per output tile, else in registers
LOWP_STAGED_PAIRS_PER_TILE = {"bf16": 16, "f16x3": 45}


def multiply_kernel(n: int, leaf: int, precision: str = "fp32", staged: bool = False) -> tuple[str, list[Path]]:
    """Name and source files (kernel file and the headers it includes) of the
    multiply kernel the timed step launches."""
    heads = [CSRC / "device.h", CSRC / "dma.h"]
    if precision != "fp32" and not staged:  # conversion in registers from the FP32 tiles
        return f"multiply_fused_kernel<{ {'bf16': 1, 'f16x3': 2}[precision] }>", [CSRC / "multiply_lowp.hip", *heads]
    if precision != "fp32":
        return f"multiply_lowp_kernel<{ {'bf16': 1, 'f16x3': 2}[precision] }>", [CSRC / "multiply_lowp.hip", *heads]
    if (leaf == 64 and n % 128 == 0) or (leaf == 128 and n % 128 == 0 and n // 128 <= 512):
        # the launch is two kernels: the multiply, then the split-tile fixup
        return "multiply_macro_dma_kernel + macro_fixup_kernel", [CSRC / "multiply_macro.hip", CSRC / "macro.h",
                                                                  *heads]
    if leaf in (32, 64):
        return f"multiply_macro_kernel<{leaf}", [CSRC / "multiply_macro.hip", CSRC / "macro.h", *heads]
    return f"multiply_kernel<{leaf}", [CSRC / "kernels.hip", CSRC / "device.h"]


def _code_only(text: str) -> str:
    """Source text without comments and blank space, so that a traffic record
    stays valid across comment and layout edits (string literals with comment
    markers do not occur in these kernel files)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def sources_sha256(sources: list[Path]) -> str:
    h = hashlib.sha256()
    for src in sources:
        h.update(_code_only(src.read_text()).encode())
    return h.hexdigest()


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse_args():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--leaf", type=int, default=64)
    ap.add_argument("--tau", type=float, default=1e-6)
    ap.add_argument("--workload", choices=["alg", "exp", "relu", "paper", "batch"], default="alg",
                    help="matrix family (default: algebraic decay); paper: the paper's evaluation matrix "
                         "0.1/(|i-j|^0.1+1) with tau from the valid-ratio search; batch: 256 independent products")
    ap.add_argument("--valid-ratio", type=float, default=0.1,
                    help="with --workload paper: the valid ratio the threshold search aims at")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-leaf", type=int, default=0, help="one leaf for every product (0: autotuned)")
    ap.add_argument("--retune", default="", help="re-run the leaf tuner and write its table to this path")
    ap.add_argument("--alpha", type=float, default=0.05, help="decay rate of --workload exp")
    ap.add_argument("--precision", choices=["fp32", "bf16", "f16x3"], default="fp32",
                    help="leaf-product precision (the mask is always the FP32 inputs')")
    ap.add_argument("--form", choices=["auto", "planes", "registers"], default="auto",
                    help="reduced precision: split planes or in-register conversion (auto: as the library picks, "
                         "from the plan's pairs per output tile)")
    ap.add_argument("--one-call", action="store_true",
                    help="time spamm_multiply as one call (fp32; leaf 32 with at most 64 tiles per side takes the "
                         "two-launch small-product path)")
    ap.add_argument("--sweep", default="1e-8,1e-4", help="other tau values timed briefly (empty: none)")
    ap.add_argument("--no-dense", action="store_true", help="skip the dense FP32 GEMM comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip timing the CPU oracle")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget for the oracle's tile sample")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/multiply_traffic.json from two rocprofv3 --pmc counter files and exit")
    ap.add_argument("--traffic-command", action="append", default=[],
                    help="with --write-traffic: the profiling commands, recorded in the file")
    return ap.parse_args()


def traffic_records() -> list[dict]:
    try:
        data = json.loads(TRAFFIC_FILE.read_text())
    except (OSError, ValueError):
        return []
    return data.get("records", []) if isinstance(data, dict) else []


def traffic_entry(kernel: str, sources: list[Path], workload: str):
    """HBM bytes per multiply launch from the committed counter summary, if it
    was taken on this kernel, its current sources and this workload (else None)."""
    sha = sources_sha256(sources)
    for rec in traffic_records():
        if rec.get("source_sha256") == sha and rec.get("kernel") == kernel and rec.get("workload") == workload:
            return rec
    return None


def _counter_rows(path: str, counter: str):
    import csv

    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") == counter:
                yield row["Kernel_Name"], float(row["Counter_Value"])


def write_traffic(fetch_csv: str, write_csv: str, args, commands: list[str]) -> int:
    """Turn two rocprofv3 --pmc runs of this script (FETCH_SIZE, then WRITE_SIZE)
    into a record of profiles/multiply_traffic.json: per-dispatch KiB of the
    multiply launch (the sum over its kernels), each scaled by what the same
    counter reads for the CALIB_BYTES device copy.  The record is keyed by the
    kernel, the workload (the same arguments as the profiled runs) and the
    kernel's sources; it replaces an older record of the same kernel and
    workload."""
    n, leaf, prec = args.n, args.leaf, args.precision
    workload = workload_name(n, leaf, args.tau, args.workload, args.alpha, prec)
    names = {name for name, _ in _counter_rows(fetch_csv, "FETCH_SIZE")}
    options = [multiply_kernel(n, leaf, prec, st) for st in ((False, True) if prec != "fp32" else (False,))]
    found = [(k, src) for k, src in options if all(any(part in nm for nm in names) for part in k.split(" + "))]
    if not found:
        print(f"{fetch_csv}: no rows of {[k for k, _ in options]}", file=sys.stderr)
        return 1
    kernel, sources = found[0]
    out = {"kernel": kernel, "workload": workload,
           "sources": [str(src.relative_to(ROOT)) for src in sources],
           "source_sha256": sources_sha256(sources), "commands": commands}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = list(_counter_rows(path, counter))
        parts = [[v for name, v in rows if part in name] for part in kernel.split(" + ")]
        copies = [v for name, v in rows if "copyBuffer" in name]
        if not all(parts) or not copies:
            print(f"{path}: no {counter} rows for {kernel} or the calibration copy", file=sys.stderr)
            return 1
        calib = max(copies)  # the CALIB_BYTES copy is the largest copy dispatch
        scale = (CALIB_BYTES / 1024.0) / calib
        key = counter.split("_")[0].lower()
        out[f"{key}_kib_per_dispatch"] = float(sum(np.mean(p) for p in parts))
        out[f"{key}_dispatches"] = min(len(p) for p in parts)
        out[f"{key}_calib_kib"] = calib
        out[f"{key}_scale"] = scale
    out["hbm_bytes_per_launch"] = round(1024.0 * (out["fetch_kib_per_dispatch"] * out["fetch_scale"]
                                                  + out["write_kib_per_dispatch"] * out["write_scale"]))
    recs = [r for r in traffic_records() if (r.get("kernel"), r.get("workload")) != (kernel, workload)]
    TRAFFIC_FILE.write_text(json.dumps({"records": recs + [out]}, indent=1) + "\n")
    print(json.dumps(out, indent=1))
    return 0


def workload_name(n: int, leaf: int, tau: float, kind: str = "alg", alpha: float = 0.05,
                  precision: str = "fp32") -> str:
    base = {
        "alg": "algebraic-decay s_ij/(1+|i-j|)^2",
        "exp": f"exponential-decay exp(-{alpha:g}|i-j|)(0.5+0.5u)",
        "relu": "ReLU-like (60% zeros, N(0,1) clipped at 0)",
        "paper": "paper matrix 0.1/(|i-j|^0.1+1) (A = B)",
    }[kind]
    name = f"{base}, N={n}, leaf {leaf}, tau={tau:g}"
    return name if precision == "fp32" else f"{name}, {precision} leaf products"


def main() -> int:
    args = parse_args()
    if args.write_traffic:
        return write_traffic(*args.write_traffic, args, args.traffic_command)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(
            f"bench.py runs on exactly one GPU (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
            "it measures the single-GPU hot path",
            file=sys.stderr,
        )
        return 2

    import torch

    from paper_2103_13042_amd import binding as sp
    from paper_2103_13042_amd import inputs

    if not torch.cuda.is_available():
        print("bench.py needs a visible GPU", file=sys.stderr)
        return 2
    dev = torch.device("cuda", 0)
    torch.backends.cuda.matmul.allow_tf32 = False

    if args.workload == "batch":
        return run_batch(args, torch, sp, inputs, dev)

    n, leaf, tau, prec = args.n, args.leaf, args.tau, args.precision
    bd = sp.bdim(n, leaf)
    log(f"generating inputs N={n} ({args.workload})")
    t0 = time.perf_counter()
    if args.workload == "alg":
        a_np, b_np = inputs.workload_alg8192(n)
        a = torch.from_numpy(a_np).to(dev)
        b = torch.from_numpy(b_np).to(dev)
    else:  # generated on the device; the CPU baseline reads them back
        if args.workload == "exp":
            a, b = inputs.exp_decay_torch(n, args.alpha, 0, dev), inputs.exp_decay_torch(n, args.alpha, 1, dev)
        elif args.workload == "paper":
            a = inputs.paper_algebraic_torch(n, dev)
            b = a.clone()
        else:
            a, b = inputs.relu_like_torch(n, 0, dev), inputs.relu_like_torch(n, 1, dev)
        a_np = b_np = None
    log(f"inputs ready in {time.perf_counter() - t0:.1f}s")
    if args.workload == "paper":  # tau for the requested valid ratio (section 3.5.2's search)
        pa, pb = sp.pyramid(a, leaf), sp.pyramid(b, leaf)
        tau, found, iters = sp.search_valid_ratio(pa, pb, n, leaf, args.valid_ratio)
        log(f"valid-ratio search: tau={tau:.6g} keeps {found} of {bd ** 3} triples "
            f"({100.0 * found / bd ** 3:.2f} %, target {100.0 * args.valid_ratio:g} %) in {iters} bisections")
        del pa, pb
    c = torch.empty_like(a)
    ws = sp.workspace(n, leaf, dev)
    bufs = sp.plan_buffers(n, leaf, dev)
    split_buf = None
    header = torch.empty(256, dtype=torch.uint8, device=dev) if prec == "f16x3" else None

    # a device-to-device copy of known size, for scaling HBM byte counters
    calib = torch.empty(CALIB_BYTES, dtype=torch.uint8, device=dev)
    calib_dst = torch.empty_like(calib)
    calib_dst.copy_(calib)
    torch.cuda.synchronize()

    # One step = the whole hot path: norms, pyramids, plan (spamm_prepare), then
    # spamm_execute as its two launch steps, so that events on the stream the
    # library launches on (torch's current stream, passed by the binding)
    # bracket the multiply kernel alone.
    # Reduced-precision products, as spamm_multiply_precision picks on the
    # device (decided here once, from the pair count of a first pass): with at
    # least 16 (BF16) or 45 (FP16 hi+lo) kept pairs per output tile on average
    # the first stage also
    # writes the split operands (spamm_prepare_split) and the multiply reads
    # them; below that the multiply converts the FP32 tiles in registers
    # (BF16: spamm_prepare_schedule, spamm_execute_bf16_scheduled; FP16 hi+lo:
    # the first stage adds the scale exponents, spamm_prepare_schedule_scales,
    # then spamm_execute_f16x3_scheduled), as spamm_multiply_precision runs it.
    staged = False
    if prec != "fp32":
        sp.prepare(a, b, tau, leaf, bufs=bufs, ws=ws)
        staged = int(bufs[2].item()) >= LOWP_STAGED_PAIRS_PER_TILE[prec] * (n // leaf) ** 2
        if args.form != "auto":
            staged = args.form == "planes"
        if staged:
            split_buf = sp.split_buffer(n, prec, dev)

    # FP32 and the in-register forms: the first stage is spamm_prepare_schedule
    # (norms, then the plan and the multiply schedule from one launch; FP16
    # hi+lo adds the scale exponents), so no schedule stage
    fused_plan = prec == "fp32" or not staged

    def stage_prepare(t):
        if prec == "f16x3" and not staged:
            return sp.prepare_scales(a, b, t, leaf, header, bufs=bufs, ws=ws, schedule=True)
        if fused_plan:
            return sp.prepare(a, b, t, leaf, bufs=bufs, ws=ws, schedule=True)
        return sp.prepare_split(a, b, t, leaf, prec, split_buf, bufs=bufs, ws=ws)

    def stage_multiply(offsets, klist):
        if prec == "fp32":
            sp.execute_scheduled(a, b, leaf, offsets, klist, c=c, ws=ws)
        elif prec == "f16x3" and not staged:
            sp.execute_f16x3(a, b, leaf, header, offsets, klist, c=c, ws=ws)
        elif prec == "bf16" and not staged:
            sp.execute_bf16(a, b, leaf, offsets, klist, c=c, ws=ws)
        else:
            sp.execute_split(split_buf, n, leaf, prec, offsets, klist, c=c, ws=ws, scheduled=True)

    one_call = args.one_call and prec == "fp32"

    def step(t):
        if one_call:
            sp.multiply(a, b, t, leaf, c=c, pairs=bufs[2], ws=ws, sync=False)
            return
        offsets, klist, _ = stage_prepare(t)
        if not fused_plan:
            sp.schedule(offsets, klist, n, leaf, ws=ws)
        stage_multiply(offsets, klist)

    def timed(t, steps, warmup):
        for _ in range(warmup):
            step(t)
        torch.cuda.synchronize()
        if one_call:  # the call's launches back to back; no stage boundaries inside it
            start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            start.record()
            for _ in range(steps):
                step(t)
            end.record()
            torch.cuda.synchronize()
            ms = start.elapsed_time(end) / steps
            return ms, [0.0, 0.0, ms], int(bufs[2].item()), ms
        # the step time: K steps back to back with no event between their
        # launches (an event record in the stream costs a few microseconds)
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(steps):
            step(t)
        end.record()
        torch.cuda.synchronize()
        plain = start.elapsed_time(end) / steps
        # then K more with events around each stage: the stage times and the
        # multiply launch's duration for the roofline
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
        start.record()
        for e in ev:
            e[0].record()
            offsets, klist, _ = stage_prepare(t)
            e[1].record()
            if not fused_plan:
                sp.schedule(offsets, klist, n, leaf, ws=ws)
            e[2].record()
            stage_multiply(offsets, klist)
            e[3].record()
        end.record()
        torch.cuda.synchronize()
        instrumented = start.elapsed_time(end) / steps
        stages = [float(np.mean([e[q].elapsed_time(e[q + 1]) for e in ev])) for q in range(3)]
        pairs = int(bufs[2].item())
        return plain, stages, pairs, instrumented

    kname, ksrc = multiply_kernel(n, leaf, prec, staged)
    if one_call:
        small = leaf == 32 and bd <= 64 and n % 4 == 0
        kname = ("spamm_multiply: leaf norms + multiply_small_kernel" if small else "spamm_multiply (all launches)")
        ksrc = None
    workload = workload_name(n, leaf, tau, args.workload, args.alpha, prec)
    # The dense FP32 GEMM the speedup is quoted against.
    d = None
    if not args.no_dense:
        for _ in range(2):
            d = torch.matmul(a, b)
        torch.cuda.synchronize()
        reps = 5
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s0.record()
        for _ in range(reps):
            d = torch.matmul(a, b)
        s1.record()
        torch.cuda.synchronize()
        dense_ms = s0.elapsed_time(s1) / reps
    # MFMA flops the multiply kernel executes per kept pair: the three FP16
    # products triple them
    flops_pair = 2.0 * leaf**3 * (3 if prec == "f16x3" else 1)
    peak = PEAK_FP32_MFMA_TFLOPS if prec == "fp32" else PEAK_F16_MFMA_TFLOPS

    # The other thresholds first, briefly.  From an idle GPU the multiply
    # kernel's first few dozen launches run up to ~25 % slower than later
    # ones while the chip's power management settles (it also slows the
    # dense GEMM's first launches); running these points first lets the
    # headline's steps run at the clock the chip sustains.
    sweep = {}
    for tok in [s for s in args.sweep.split(",") if s.strip()]:
        t = float(tok)
        ms, (_, _, em), p, _ = timed(t, max(5, args.steps // 2), 2)
        sweep[f"{t:g}"] = {
            "ms_per_step": round(ms, 4),
            "dense_equiv_tflops": round(2.0 * n**3 / (ms * 1e-3) / 1e12, 3),
            "multiply_ms": round(em, 4),
            "mfma_frac": round(flops_pair * p / (em * 1e-3) / 1e12 / peak, 4) if p else None,
            "pairs": p,
        }
        log(f"tau={t:g}: {ms:.3f} ms/step, pairs {p}")

    log(f"warmup {args.warmup}, timing {args.steps} steps at tau={tau:g}")
    ms_step, (prep_ms, sched_ms, kern_ms), pairs, ms_instr = timed(tau, args.steps, args.warmup)
    dense_equiv = 2.0 * n**3 / (ms_step * 1e-3) / 1e12
    flops_mul = flops_pair * pairs
    achieved = flops_mul / (kern_ms * 1e-3) / 1e12
    log(f"{ms_step:.3f} ms/step (prepare {prep_ms:.3f}, schedule {sched_ms:.3f}, {kname} {kern_ms:.3f}), "
        f"pairs {pairs}, {dense_equiv:.1f} dense-equiv TFLOP/s, multiply {achieved:.1f} TFLOP/s")

    result = {
        "metric": METRIC,
        "value": round(dense_equiv, 3),
        "unit": "TFLOP/s (dense-equivalent 2N^3/t)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16 products, f32 accumulate", "f16x3": "f16 hi+lo products, f32 accumulate"}[prec],
        "data": "synthetic",
        "config": {
            "workload": workload,
            "n": n,
            "leaf": leaf,
            "tau": tau,
            "precision": prec,
            "form": ("fp32" if prec == "fp32" else "split planes" if staged else "in registers"),
            "pairs": pairs,
            "valid_ratio": pairs / bd**3,
        },
        "stages_ms": {"prepare": round(prep_ms, 4), "schedule": round(sched_ms, 4), "multiply": round(kern_ms, 4)},
    }
    if fused_plan:  # spamm_prepare_schedule: the schedule comes with the plan
        result["stages_ms"] = {"prepare_schedule": round(prep_ms, 4), "multiply": round(kern_ms, 4)}
    # the step time of the event-instrumented pass the stages come from
    result["stages_ms"]["step_with_stage_events"] = round(ms_instr, 4)
    result["timing"] = (f"after the tau sweep: {args.warmup} warm-up steps, {args.steps} steps back to back "
                        f"(ms_per_step), then {args.steps} steps with an event around each stage (stages_ms, "
                        "roofline.ms_per_launch)")
    if one_call:
        result["stages_ms"] = {"spamm_multiply": round(ms_step, 4)}
        result["config"]["entry"] = "spamm_multiply"
        result["timing"] = (f"after the tau sweep: {args.warmup} warm-up calls, {args.steps} calls back to back "
                            "(ms_per_step and roofline.ms_per_launch)")

    tr = traffic_entry(kname, ksrc, workload) if ksrc else None
    result["roofline"] = {
        "bound": "mfma",
        "kernel": kname,
        "flop_per_launch": flops_mul,
        "ms_per_launch": round(kern_ms, 4),
        "achieved": round(achieved, 3),
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": round(achieved / peak, 4),
        "traffic": tr["hbm_bytes_per_launch"] if tr else None,
    }
    if one_call:
        result["roofline"]["note"] = "ms_per_launch is the whole call (every launch of spamm_multiply)"

    # approximation + precision against the dense FP32 product (which was
    # timed before the steps)
    if d is not None:
        rel = float(torch.linalg.norm(c.double() - d.double()) / torch.linalg.norm(d.double()))
        result["dense_gemm"] = {
            "library": f"torch.matmul fp32 (torch {torch.__version__}, TF32 off)",
            "ms": round(dense_ms, 4),
            "tflops": round(2.0 * n**3 / (dense_ms * 1e-3) / 1e12, 3),
        }
        result["speedup_vs_dense"] = round(dense_ms / ms_step, 3)
        result["rel_err_vs_dense_fp32"] = rel
        log(f"dense {dense_ms:.3f} ms, speedup {dense_ms / ms_step:.2f}x, rel err vs dense {rel:.2e}")
        del d

    if sweep:
        result["tau_sweep"] = sweep

    if not args.no_cpu_baseline:
        if a_np is None:
            a_np, b_np = a.cpu().numpy(), b.cpu().numpy()
        # the oracle computes the FP32 inputs' SpAMM in FP64: with reduced
        # precision the sampled difference is that form's error
        result["cpu_baseline"], result["rel_err_vs_oracle_sampled"] = cpu_baseline(
            a_np, b_np, c.cpu().numpy(), tau, leaf, args.cpu_seconds
        )

    print(json.dumps(result), flush=True)
    return 0


def run_batch(args, torch, sp, inputs, dev) -> int:
    """Batched form: `--batch-count` products, n log-uniform in [256, 4096],
    exponential decay with rates uniform in [0.01, 0.5), tau; leaves from the
    autotuner.  Times a per-product loop of spamm_multiply, the batched entry
    point run eagerly, and the batch captured in a graph and replayed."""
    from paper_2103_13042_amd import autotune

    tau = args.tau
    specs = inputs.batch_specs(args.batch_count)
    log(f"batch of {len(specs)}: generating inputs")
    a_l = [inputs.exp_decay_torch(n, aa, sa, dev) for n, aa, _, sa, _ in specs]
    b_l = [inputs.exp_decay_torch(n, ab, sb, dev) for n, _, ab, _, sb in specs]
    if args.batch_leaf:
        leaves, table = [args.batch_leaf] * len(specs), None
    else:
        t0 = time.perf_counter()
        if autotune.TABLE_FILE.exists() and not args.retune:
            log(f"leaf sizes from {autotune.TABLE_FILE.name}")
            table = autotune.load(autotune.TABLE_FILE)
        else:
            log("autotuning leaf sizes")
            table = autotune.tune(dev, tau=tau)
            if args.retune:
                autotune.save(table, args.retune)
        tune_s = time.perf_counter() - t0
        leaves = [autotune.choose(table, n, autotune.density(a, b, tau))
                  for (n, *_), a, b in zip(specs, a_l, b_l)]
    bt = sp.Batch(a_l, b_l, leaves, [tau] * len(specs))
    dense_flop = sum(2.0 * n**3 for n, *_ in specs)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    # per-product loop: the single-product entry point, one product after another
    loop_ws = {}
    loop_c = [torch.empty_like(a) for a in a_l]
    loop_pairs = torch.empty(len(specs), dtype=torch.int64, device=dev)

    def loop():
        for q, (a, b) in enumerate(zip(a_l, b_l)):
            key = (a.shape[0], leaves[q])
            if key not in loop_ws:
                loop_ws[key] = sp.workspace(key[0], key[1], dev).clone()
            sp.multiply(a, b, tau, leaves[q], c=loop_c[q], pairs=loop_pairs[q:q + 1], ws=loop_ws[key], sync=False)

    steps = max(3, args.steps // 4)
    log("timing the per-product loop")
    loop_ms = timed(loop, steps, 2)
    log("timing the batched launch (eager)")
    eager_ms = timed(bt.run, args.steps, args.warmup)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bt.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bt.run()
    log("timing graph replays")
    graph_ms = timed(g.replay, args.steps, args.warmup)
    pairs = bt.pairs.cpu().tolist()
    if pairs != loop_pairs.cpu().tolist():
        log("pairs differ between the batch and the loop")
        return 1
    rel = max(float(torch.linalg.norm((x - y).double()) / max(float(torch.linalg.norm(y.double())), 1e-300))
              for x, y in zip(bt.c, loop_c))
    mul_flop = sum(2.0 * leaves[q] ** 3 * pairs[q] for q in range(len(specs)))
    value = dense_flop / (graph_ms * 1e-3) / 1e12
    hist = {str(L): leaves.count(L) for L in sorted(set(leaves))}
    log(f"loop {loop_ms:.3f} ms, batched eager {eager_ms:.3f} ms, graph {graph_ms:.3f} ms; leaves {hist}")
    achieved = mul_flop / (graph_ms * 1e-3) / 1e12
    result = {
        "metric": METRIC, "value": round(value, 3), "unit": "TFLOP/s (dense-equivalent sum of 2N^3 / t)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(graph_ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batch of {len(specs)} products, n log-uniform in [256, 4096], exponential decay "
                               f"rates U[0.01, 0.5), tau={tau:g}, autotuned leaves",
                   "form": "each stage one launch over the whole batch (about 11 launches, one persistent multiply "
                           "per leaf class) captured in one graph and replayed; not one persistent launch",
                   "products": len(specs), "tau": tau, "leaves": hist, "pairs": int(sum(pairs)),
                   "dense_equiv_flop": dense_flop},
        "stages_ms": {"per_product_loop": round(loop_ms, 4), "batched_eager": round(eager_ms, 4),
                      "batched_graph": round(graph_ms, 4)},
        "speedup_vs_loop": round(loop_ms / graph_ms, 3),
        "rel_diff_batch_vs_loop": rel,
        "roofline": {"bound": "mfma", "kernel": "whole batched run (every stage)", "flop_per_launch": mul_flop,
                     "ms_per_launch": round(graph_ms, 4), "achieved": round(achieved, 3),
                     "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_MFMA_TFLOPS, 4),
                     "traffic": None},
    }
    if table is not None:
        result["autotune"] = {"seconds": round(tune_s, 2), "buckets": table["buckets"]}
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline_batch(a_l, b_l, leaves, tau, specs, args.cpu_seconds)
    print(json.dumps(result), flush=True)
    return 0


def cpu_baseline_batch(a_l, b_l, leaves, tau, specs, budget_s):
    """The FP64 oracle over whole products in a seeded order until the budget
    is spent; the rate is their dense-equivalent flops over the time."""
    import oracle

    oracle.use_native_build()  # -O3 -march=native, compiled on this host
    order = np.random.default_rng(77).permutation(len(specs))
    done, flop, t_all = 0, 0.0, 0.0
    for q in order:
        a, b = a_l[q].cpu().numpy(), b_l[q].cpu().numpy()
        t0 = time.perf_counter()
        oracle.spamm(a, b, tau, leaves[q])
        t_all += time.perf_counter() - t0
        flop += 2.0 * a.shape[0] ** 3
        done += 1
        if t_all >= budget_s:
            break
    return {"value": flop / t_all / 1e12, "unit": "TFLOP/s (dense-equivalent sum of 2N^3 / t)",
            "cores": oracle.max_threads(), "kind": "oracle", "cpu": host_cpu(),
            "sample": f"FP64 oracle on {done} of {len(specs)} products (whole products, seeded order), {t_all:.1f}s"}


def host_cpu() -> str:
    """The host CPU's model name (from /proc/cpuinfo), for the CPU-baseline record."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(a_np, b_np, c_gpu, tau, leaf, budget_s):
    """Time the FP64 oracle on the host cores over the same workload: whole
    passes (both pyramids, then every output tile, in a seeded random order)
    until the time budget is spent.  If the first pass alone outruns the
    budget, it stops there and its time is extrapolated from the tile rate.
    Also compares the GPU result with the oracle on the tiles of that pass."""
    import oracle

    build = oracle.use_native_build()  # -O3 -march=native, compiled on this host
    n = a_np.shape[0]
    bd = oracle.bdim(n, leaf)
    total = bd * bd
    log(f"cpu baseline: oracle ({build.name}) on {oracle.max_threads()} threads, budget {budget_s:.0f}s")
    order = np.random.default_rng(1234).permutation(total)
    chunk = 256
    times, num, den = [], 0.0, 0.0
    partial = None
    while not times or sum(times) < budget_s:
        t0 = time.perf_counter()
        pa, pb = oracle.pyramid(a_np, leaf), oracle.pyramid(b_np, leaf)
        t_pyr = time.perf_counter() - t0
        done, t_tiles = 0, 0.0
        while done < total:
            if not times and t_pyr + t_tiles > budget_s:
                break
            ids = order[done : done + chunk]
            tiles = np.stack([ids // bd, ids % bd], axis=1)
            t1 = time.perf_counter()
            ct, _, _ = oracle.spamm_tiles(a_np, b_np, tau, leaf, tiles, pyr_a=pa, pyr_b=pb)
            t_tiles += time.perf_counter() - t1
            if not times:
                for t, (i, j) in enumerate(tiles):
                    r1, c1 = min(n, (i + 1) * leaf), min(n, (j + 1) * leaf)
                    blk = c_gpu[i * leaf : r1, j * leaf : c1].astype(np.float64)
                    ref = ct[t, : r1 - i * leaf, : c1 - j * leaf]
                    num += float(np.sum((blk - ref) ** 2))
                    den += float(np.sum(ref**2))
            done += len(ids)
        if done < total:  # first pass over budget: extrapolate it
            partial = (done, t_pyr + t_tiles)
            times.append(t_pyr + t_tiles * total / done)
            break
        times.append(t_pyr + t_tiles)
    t_pass = float(np.median(times))
    value = 2.0 * n**3 / t_pass / 1e12
    rel = math.sqrt(num / den) if den > 0 else math.sqrt(num)
    if partial:
        sample = (f"FP64 oracle: pyramids of A and B, then {partial[0]} of {total} output tiles in seeded random "
                  f"order ({partial[1]:.1f}s), extrapolated to all tiles ({t_pass:.1f}s)")
    else:
        sample = (f"FP64 oracle, the whole workload (pyramids of A and B, then all {total} output tiles) "
                  f"repeated {len(times)} times in {sum(times):.1f}s; median {t_pass:.3f}s per pass")
    log(f"cpu baseline: {sample}")
    return (
        {"value": value, "unit": "TFLOP/s (dense-equivalent 2N^3/t)", "cores": oracle.max_threads(),
         "kind": "oracle", "cpu": host_cpu(), "build": "gcc -O3 -march=native -fopenmp", "sample": sample},
        rel,
    )


if __name__ == "__main__":
    sys.exit(main())
