"""Host-side logic of bench.py (no GPU): the one-GPU contract, and the
rocprofv3 counter ingestion that gives the roofline's `traffic` (counters
scaled by a plain copy of known size, keyed by the kernel-source hash, so
that a changed kernel reports no traffic figure until it is measured)."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_counter_ingestion_and_hash_key(tmp_path, monkeypatch):
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    stage = "void ssd::k_stage<4, true, false, false, false>(...)"
    copy = "__amd_rocclr_copyBuffer"
    # a plain copy of 1 GiB: FETCH_SIZE (KiB) shows half the bytes read,
    # WRITE_SIZE (KiB) all the bytes written
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE", [(stage, 100000.0), (stage, 300000.0),
                                                    ("void ssd::k_mortar<4, false>(...)", 5.0)])
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE", [(stage, 50000.0)])
    _counter_csv(tmp_path / "cf.csv", "FETCH_SIZE", [(copy, (1 << 30) / 2 / 1024)])
    _counter_csv(tmp_path / "cw.csv", "WRITE_SIZE", [(copy, (1 << 30) / 1024)])
    bench.ingest_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"),
                          str(tmp_path / "cf.csv"), str(tmp_path / "cw.csv"), E=1000, N=4)
    rec = json.loads(out.read_text())
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["fetch_bytes_per_launch"] == pytest.approx(200000.0 * 1024 * 2.0)   # mean of the stage launches
    assert rec["write_bytes_per_launch"] == pytest.approx(50000.0 * 1024)
    assert rec["kernel_hash"] == bench.kernel_hash()
    assert bench.traffic_for(bench.kernel_hash(), 1000, 4) == pytest.approx(rec["bytes_per_launch"])
    # another source hash, size or order gives no traffic figure
    assert bench.traffic_for("0" * 16, 1000, 4) is None
    assert bench.traffic_for(bench.kernel_hash(), 999, 4) is None
    assert bench.traffic_for(bench.kernel_hash(), 1000, 3) is None

