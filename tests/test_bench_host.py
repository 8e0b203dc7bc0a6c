"""Host-side parts of bench.py (no GPU): the HBM-traffic calibration written to
profiles/traffic.json and read back by the bench line, and the single-GPU exit."""
import csv
import json
import os
import subprocess
import sys

import bench


def _counter_csv(path, counter, copy_kib, kernels):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        w.writerow({"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": counter,
                    "Counter_Value": 3.0})  # a small upload: not the probe
        w.writerow({"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": counter,
                    "Counter_Value": copy_kib})
        for name, v in kernels:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})


def test_traffic_calibration(tmp_path, monkeypatch):
    """Each counter is scaled by what it reads for the 1 GiB copy probe: FETCH_SIZE reads
    half the probe's KiB, WRITE_SIZE all of them; the kernel's per-launch bytes are the
    median over its launches, keyed by the kernel source hash."""
    probe_kib = bench.COPY_PROBE_BYTES / 1024
    f = tmp_path / "fetch.csv"
    w = tmp_path / "write.csv"
    k = "void gp::k_p2pmix_pre<4, 1>(gp::RefineArgs, int)"
    _counter_csv(f, "FETCH_SIZE", probe_kib / 2, [(k, 100.0), (k, 300.0), (k, 200.0)])
    _counter_csv(w, "WRITE_SIZE", probe_kib, [(k, 50.0), (k, 50.0), (k, 70.0)])
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    bench.write_traffic(str(f), str(w))
    t = json.load(open(out))["k_p2pmix_pre"]
    assert t["copy_factor_fetch"] == 0.5 and t["copy_factor_write"] == 1.0
    assert t["fetch_bytes_per_launch"] == 200.0 * 1024 / 0.5
    assert t["write_bytes_per_launch"] == 50.0 * 1024
    assert t["launches"] == 3 and t["kernel_source_sha"] == bench.kernel_hash()
    assert bench.load_traffic("k_p2pmix_pre", bench.WORKLOAD_NAME) == t["hbm_bytes_per_launch"]
    assert bench.load_traffic("k_p2pmix_pre", "another workload") is None
    # a kernel source that changed since the counters were taken gives no figure
    monkeypatch.setattr(bench, "kernel_hash", lambda: "0" * 16)
    assert bench.load_traffic("k_p2pmix_pre", bench.WORKLOAD_NAME) is None


def test_more_than_one_gpu_exits():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
