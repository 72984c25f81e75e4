"""Host-side parts of bench.py (no GPU): the one-GPU guard, the traffic record
built from rocprofv3 counter files, and what invalidates that record."""

from __future__ import annotations

import json
import subprocess
import sys
import types
from pathlib import Path

import bench

ROOT = Path(__file__).resolve().parents[1]


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr


def _counter_csv(path: Path, counter: str, rows):
    head = "Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n"
    path.write_text(head + "".join(f'{i},"{k}",{counter},{v}\n' for i, (k, v) in enumerate(rows)))


def test_traffic_record_scales_each_counter_by_the_calibration_copy(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", tmp_path / "traffic.json")
    calib_kib = bench.CALIB_BYTES / 1024
    mul = "spamm::multiply_macro_dma_kernel(float const*, ...)"
    fix = "spamm::macro_fixup_kernel(float*, ...)"
    # the copy reads half its bytes in FETCH_SIZE units (factor 2), writes all
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE", [("__amd_rocclr_copyBuffer", calib_kib / 2),
                                                    ("__amd_rocclr_copyBuffer", 4.0), (mul, 1000.0), (mul, 1200.0),
                                                    (fix, 50.0), (fix, 50.0)])
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", calib_kib), (mul, 300.0),
                                                    (mul, 300.0), (fix, 20.0), (fix, 20.0)])
    args = types.SimpleNamespace(n=8192, leaf=64, tau=1e-6, workload="alg", alpha=0.05, precision="fp32")
    assert bench.write_traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), args, ["cmd"]) == 0
    recs = json.loads((tmp_path / "traffic.json").read_text())["records"]
    assert len(recs) == 1
    rec = recs[0]
    assert rec["kernel"] == "multiply_macro_dma_kernel + macro_fixup_kernel"
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    # per launch: (mean 1100 + 50) KiB read x 2, (300 + 20) KiB written x 1
    assert rec["hbm_bytes_per_launch"] == round(1024 * ((1100 + 50) * 2 + (300 + 20)))
    k, src = bench.multiply_kernel(8192, 64)
    assert bench.traffic_entry(k, src, bench.workload_name(8192, 64, 1e-6)) == rec
    assert bench.traffic_entry(k, src, bench.workload_name(8192, 64, 1e-8)) is None  # another workload
    # a second workload adds a record; the same workload again replaces its own
    args.tau = 1e-8
    assert bench.write_traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), args, ["cmd"]) == 0
    assert bench.write_traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), args, ["cmd"]) == 0
    assert len(json.loads((tmp_path / "traffic.json").read_text())["records"]) == 2
    assert bench.traffic_entry(k, src, bench.workload_name(8192, 64, 1e-6)) == rec


def test_traffic_record_key_ignores_comments_but_not_code():
    a = "int f(int x) { // twice\n  return 2 * x; /* doubled */ }\n"
    b = "int f(int x) {\n\n  return 2 * x;   }  // edited comment\n"
    c = "int f(int x) { return 3 * x; }\n"
    assert bench._code_only(a) == bench._code_only(b) != bench._code_only(c)
