"""Host-side logic of bench.py (no GPU): the reduction of rocprofv3 counter files to
HBM bytes per launch, and the one-GPU guard."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _counters(path, counter, rows):
    cols = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for i, (name, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_traffic_summary_scales_by_the_copy_probe(tmp_path):
    import bench

    probe = "void at::native::vectorized_elementwise_kernel<4, float>(...)"
    mix = "void tt::(anonymous namespace)::mix_kernel<float, 2, false>(int4 const*, ...)"
    other = "void tt::(anonymous namespace)::mix_kernel<float, 1, false>(int4 const*, ...)"
    # the probe reads 1 GiB but the read counter shows half of it; writes are counted in full
    _counters(tmp_path / "f.csv", "FETCH_SIZE", [(probe, 524288.0), (probe, 10.0), (mix, 1000.0), (mix, 3000.0),
                                                (other, 50.0)])
    _counters(tmp_path / "w.csv", "WRITE_SIZE", [(probe, 1048576.0), (mix, 500.0), (mix, 1500.0), (other, 20.0)])
    run = {"config": {"workload": "w"}, "kernels": {
        "mix2_gather": {"ms": 2.0, "launches": 2, "gbs": 4.096},      # 4.096e6 bytes per launch
        "mix1_gather": {"ms": 1.0, "launches": 1, "gbs": 1.0}}}
    (tmp_path / "r.json").write_text("log line\n" + json.dumps(run) + "\n")
    t = bench.traffic_summary(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "r.json"), ["c"])
    assert t["copy_probe"]["read_scale"] == 2.0 and t["copy_probe"]["write_scale"] == 1.0
    assert t["read_counters"] == ["FETCH_SIZE"]
    k = t["kernels"]["mix2_gather"]
    assert k["launches_counted"] == 2
    assert k["hbm_read_bytes_per_launch"] == 2000 * 1024 * 2
    assert k["hbm_write_bytes_per_launch"] == 1000 * 1024
    assert k["hbm_bytes_per_launch"] == 2000 * 1024 * 2 + 1000 * 1024
    assert k["algorithmic_bytes_per_launch"] == 4096000
    assert set(t["kernels"]) == {"mix2_gather", "mix1_gather"}
    assert t["source_sha256_16"] == bench.kernel_source_hash()


def _raw_reads(path, rows):
    """rows: (kernel, n_requests, n_32B, n_128B) per dispatch, one counter per CSV row"""
    cols = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for i, (name, n, n32, n128) in enumerate(rows):
            for c, v in (("TCC_EA0_RDREQ_sum", n), ("TCC_EA0_RDREQ_32B_sum", n32),
                         ("TCC_EA0_RDREQ_128B_sum", n128), ("TCC_BUBBLE_sum", 0)):
                w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": c, "Counter_Value": v})


def test_traffic_summary_from_read_request_counters(tmp_path):
    import bench

    probe = "void at::native::vectorized_elementwise_kernel<4, float>(...)"
    mix = "void tt::(anonymous namespace)::mix_kernel<float, 2, false>(int4 const*, ...)"
    # the probe's 1 GiB arrives as 2^23 requests of 128 bytes: scale exactly 1
    _raw_reads(tmp_path / "r.csv", [(probe, 1 << 23, 0, 1 << 23), (mix, 100, 10, 40), (mix, 300, 30, 120)])
    _counters(tmp_path / "w.csv", "WRITE_SIZE", [(probe, 1048576.0), (mix, 1.0), (mix, 3.0)])
    run = {"config": {"workload": "w"}, "kernels": {"mix2_gather": {"ms": 2.0, "launches": 2, "gbs": 1.0}}}
    (tmp_path / "j.json").write_text(json.dumps(run) + "\n")
    t = bench.traffic_summary(str(tmp_path / "r.csv"), str(tmp_path / "w.csv"), str(tmp_path / "j.json"), [])
    assert t["copy_probe"]["read_scale"] == 1.0 and t["copy_probe"]["write_scale"] == 1.0
    assert t["read_counters"][0] == "TCC_EA0_RDREQ_sum"
    k = t["kernels"]["mix2_gather"]
    # per dispatch 128 N128 + 32 N32 + 64 (N - N128 - N32), averaged over the two dispatches
    b1 = 128 * 40 + 32 * 10 + 64 * 50
    assert k["hbm_read_bytes_per_launch"] == (b1 + 3 * b1) // 2
    assert k["hbm_write_bytes_per_launch"] == 2 * 1024


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_measured_traffic_requires_the_current_kernel_sources(tmp_path, monkeypatch):
    import bench

    rec = {"hbm_bytes_per_launch": 3000, "traffic_over_algorithmic": 1.5}
    f = tmp_path / "t.json"
    f.write_text(json.dumps({"source_sha256_16": bench.kernel_source_hash(), "kernels": {"mix2_gather": rec}}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("mix2_gather") == rec
    assert bench.measured_traffic("gemm_R") is None
    f.write_text(json.dumps({"source_sha256_16": "0" * 16, "kernels": {"mix2_gather": rec}}))
    assert bench.measured_traffic("mix2_gather") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic("mix2_gather") is None


def test_stats_summary_puts_profiler_and_event_timing_side_by_side(tmp_path):
    import bench

    cols = ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"]
    with open(tmp_path / "s.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=cols)
        w.writeheader()
        w.writerow({"Name": "void tt::(anonymous namespace)::mix_kernel<float, 2, false>(int4 const*)", "Calls": 4,
                    "TotalDurationNs": 4.0e6, "AverageNs": 1.0e6, "Percentage": 80, "MinNs": 0, "MaxNs": 0,
                    "StdDev": 0})
        w.writerow({"Name": "tt::fill_kernel(unsigned int*, unsigned long)", "Calls": 10, "TotalDurationNs": 1.0e6,
                    "AverageNs": 1.0e5, "Percentage": 20, "MinNs": 0, "MaxNs": 0, "StdDev": 0})
    run = {"value": 2.5, "matvecs_per_sweep": 4,
           "config": {"workload": "w", "L": 8, "chi": 16, "subdomains": [4, 4], "matvec": "f32",
                      "concurrent_subdomain_solves": 1},
           "kernels": {"mix2_gather": {"ms": 4.2, "launches": 4}},
           "roofline": {"kernel": "mix2_gather", "avg_launch_us": 1050.0, "bound": "hbm", "achieved": 1.0,
                        "peak": 8000.0, "unit": "GB/s", "frac": 0.000125}}
    (tmp_path / "r.json").write_text(json.dumps(run) + "\n")
    text = bench.stats_summary(str(tmp_path / "s.csv"), str(tmp_path / "r.json"), "the command")
    assert "command: the command" in text
    assert bench.kernel_source_hash() in text
    line = [ln for ln in text.splitlines() if ln.strip().startswith("mix2_gather")][0]
    assert "1050.0 us/launch" in line and "rocprofv3   1000.0 us/launch" in line
    assert "total kernel time 0.005 s over 14 dispatches" in text
