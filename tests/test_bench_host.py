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
    assert t["copy_probe"]["fetch_scale"] == 2.0 and t["copy_probe"]["write_scale"] == 1.0
    k = t["kernels"]["mix2_gather"]
    assert k["launches_counted"] == 2
    assert k["hbm_read_bytes_per_launch"] == 2000 * 1024 * 2
    assert k["hbm_write_bytes_per_launch"] == 1000 * 1024
    assert k["hbm_bytes_per_launch"] == 2000 * 1024 * 2 + 1000 * 1024
    assert k["algorithmic_bytes_per_launch"] == 4096000
    assert set(t["kernels"]) == {"mix2_gather", "mix1_gather"}
    assert t["source_sha256_16"] == bench.kernel_source_hash()


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
