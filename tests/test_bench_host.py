"""Host-side logic of the benchmark (no GPU): the one-GPU guard, the names
of the timed kernels, and the lookup of measured HBM traffic, which the
benchmark reports only for the kernel variant, launch length and kernel
sources the counters were taken on."""
import hashlib
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_kernel_names():
    reg = {"coef_mode": 3, "block_threads": 64, "reg_slots": 2, "reg_len": 8, "syn_hbm": 0}
    assert bench.kernel_name(reg) == "reg_step_kernel<64, 2, 8, false>"
    assert bench.kernel_name(dict(reg, block_threads=128, reg_slots=1, syn_hbm=1)) == "reg_step_kernel<128, 1, 8, true>"
    assert bench.kernel_name({"coef_mode": 1, "block_threads": 256}) == "step_kernel<256, true>"
    assert bench.kernel_name({"coef_mode": 2, "block_threads": 64}) == "step_kernel<64, false>"


def test_measured_traffic_only_for_the_profiled_kernel(tmp_path):
    src = tmp_path / "kernel.hip"
    src.write_bytes(b"__global__ void k() {}\n")
    kern = "reg_step_kernel<64, 2, 8, false>"
    rec = {"kernel_sources": [str(src)], "kernel_sha256": hashlib.sha256(src.read_bytes()).hexdigest(),
           "kernel": kern, "fixed_bytes_per_launch": 3.0e8, "bytes_per_step": 1.0e6}
    path = tmp_path / "traffic.txt"
    path.write_text(json.dumps({"config2": rec}))
    # a launch of any length: the fixed part plus the per-step part
    assert bench.measured_traffic(str(path), 2, kern, 200.0) == 3.0e8 + 2.0e8
    assert bench.measured_traffic(str(path), 2, kern, 20.0) == 3.0e8 + 2.0e7
    assert bench.measured_traffic(str(path), 2, "reg_step_kernel<128, 2, 8, false>", 200.0) is None
    assert bench.measured_traffic(str(path), 5, kern, 200.0) is None
    assert bench.measured_traffic(str(tmp_path / "missing.txt"), 2, kern, 200.0) is None
    src.write_bytes(b"__global__ void k() { }\n")  # the kernel changed since
    assert bench.measured_traffic(str(path), 2, kern, 200.0) is None


def test_committed_traffic_records_name_existing_sources():
    recs = json.load(open(os.path.join(ROOT, "profiles", "traffic.txt")))
    assert "config2" in recs
    for name, rec in recs.items():
        if not name.startswith("config"):
            continue
        assert rec["kernel"].startswith(("reg_step_kernel<", "step_kernel<"))
        if "bytes_per_step" in rec:
            assert rec["fixed_bytes_per_launch"] >= 0 and rec["bytes_per_step"] > 0, name
        else:  # a record of one launch length (not used by the benchmark)
            assert rec["bytes_per_launch"] > 0, name
        for p in rec["kernel_sources"]:
            assert os.path.exists(os.path.join(ROOT, p)), p


def test_timed_window_is_whole_epochs():
    """The benchmark rounds its timed steps and its warm-up up to whole
    epochs (at least one warm-up epoch), so the exchange is always timed."""
    src = open(os.path.join(ROOT, "bench.py")).read()
    assert "warmup = max(1, -(-args.warmup // K)) * K" in src
    assert "steps = max(1, -(-args.steps // K)) * K" in src
