"""Host-side checks of bench.py's contract (no GPU): more than one GPU is refused with a
message, the algorithmic flop count of the headline is the Cholesky's, and the committed
HBM-traffic record is used only while it matches the kernel source it was measured on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_cholesky_flop_count():
    # n^3/3 + n^2/2 + n/6: the flops of the textbook column Cholesky (n = 1: one square root)
    assert bench.chol_flops(1) == pytest.approx(1.0)
    assert bench.chol_flops(3) == pytest.approx(9 + 4.5 + 0.5)


def test_traffic_record_tracks_the_kernel_source(tmp_path, monkeypatch):
    with open(bench.TRAFFIC_RECORD) as f:
        rec = json.load(f)
    kernel = "gemm_trace_kernel<double, 3>"
    assert rec["bytes_per_launch"][kernel] > 0
    assert bench.kernel_family(kernel) == "f64_f32" and bench.kernel_family("gemm_bf16x_t256_kernel<6>") == "bf16"
    src = tmp_path / "gemm.hip"
    src.write_text("// another kernel source\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", {"f64_f32": [str(src)], "bf16": [str(src)]})
    assert bench.recorded_traffic(kernel) is None
    fam = rec["source_families"]["f64_f32"]
    monkeypatch.setattr(bench, "KERNEL_SOURCES", {"f64_f32": [os.path.join(ROOT, f) for f in fam["files"]], "bf16": []})
    if bench.source_digest(bench.KERNEL_SOURCES["f64_f32"]) == fam["sha256_16"]:
        assert bench.recorded_traffic(kernel) == rec["bytes_per_launch"][kernel]
