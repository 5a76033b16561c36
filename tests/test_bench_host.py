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
        assert rec["kernel"].startswith(("reg_step_kernel<", "step_kernel<", "var_step_kernel<"))
        if "bytes_per_step" in rec:
            # a kernel that streams nothing per step fits a per-step term of
            # counter noise, which may come out slightly negative
            fixed, per_step = rec["fixed_bytes_per_launch"], rec["bytes_per_step"]
            assert fixed > 0 and per_step >= -1e-4 * fixed, name
            assert all(fixed + per_step * k > 0 for k in rec["epoch_lengths"]), name
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


def test_fit_traffic_recovers_fixed_and_per_step_bytes(tmp_path):
    """The traffic fit from counter runs at two epoch lengths: the step
    kernels' FETCH_SIZE and WRITE_SIZE (KiB, summed over every launch class
    and divided by the epochs run) scaled by what the counters read for the
    2 GiB copy, then bytes per epoch = fixed + per_step K solved exactly."""
    import csv
    import json
    import bench
    fixed, per_step, sf, sw = 4.0e8, 6.0e3, 2.0, 1.0  # bytes, bytes, KiB -> x scale
    for K in (100, 200):
        epochs = 9 * 200 // K
        (tmp_path / f"bench_K{K}.json").write_text(json.dumps({"steps": 8 * 200, "warmup": 200}) + "\n")
        per_epoch = fixed + per_step * K
        for sub, ctr, scale, share in (("fetch", "FETCH_SIZE", sf, 0.75), ("write", "WRITE_SIZE", sw, 0.25)):
            d = tmp_path / f"{sub}_K{K}"
            d.mkdir()
            with open(d / "run_counter_collection.csv", "w", newline="") as f:
                w = csv.writer(f)
                w.writerow(["Kernel_Name", "Counter_Name", "Counter_Value"])
                for _ in range(epochs):  # two launch classes per epoch
                    kib = per_epoch * share / scale / 1024.0
                    w.writerow(["void reg_step_kernel<256, 1, 8>(x)", ctr, 0.25 * kib])
                    w.writerow(["void reg_step_kernel<256, 2, 8>(x)", ctr, 0.75 * kib])
                for _ in range(10):
                    w.writerow(["__amd_rocclr_copyBuffer", ctr, 2097152.0 / scale])
                w.writerow(["__amd_rocclr_copyBuffer", ctr, 12.0])
    out = tmp_path / "traffic.json"
    rec = bench.fit_traffic(str(tmp_path), "config3", "reg_step_kernel<256, 3, 8, true>", "reg", str(out))
    assert abs(rec["fetch_scale"] - sf) < 1e-12 and abs(rec["write_scale"] - sw) < 1e-12
    assert abs(rec["fixed_bytes_per_launch"] - fixed) < 1e-3 and abs(rec["bytes_per_step"] - per_step) < 1e-6
    got = bench.measured_traffic(str(out), 3, "reg_step_kernel<256, 3, 8, true>", 1000)
    assert abs(got - (fixed + 1000 * per_step)) < 1e-2
    assert bench.measured_traffic(str(out), 3, "reg_step_kernel<256, 2, 8, true>", 1000) is None
