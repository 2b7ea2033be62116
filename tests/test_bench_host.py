"""Host logic of bench.py (CPU): the one-GPU guard, the traffic figure taken
from rocprofv3 counter files (scaled by a plain copy's reading, tied to the
kernel sources it was measured on), percentiles and the limiter note."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

MARCH = "void rtv::(anonymous namespace)::march_batch_kernel<6, 0, false>(char*, rtv::LaunchShape, int, int)"
COPY = "__amd_rocclr_copyBuffer"


def _counters(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (k, c, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_ingest_traffic_scales_by_the_copy_and_takes_medians(tmp_path, monkeypatch):
    d = tmp_path / "prof"
    # a 1 GiB copy reads as 2^19 KiB fetched (half the bytes) and 2^20 KiB written
    _counters(str(d / "copy_fetch" / "c_counter_collection.csv"), [(COPY, "FETCH_SIZE", 1 << 19)])
    _counters(str(d / "copy_write" / "c_counter_collection.csv"), [(COPY, "WRITE_SIZE", 1 << 20)])
    # three marcher dispatches: the medians are taken (an outlier first)
    _counters(str(d / "fetch" / "o_counter_collection.csv"),
              [(MARCH, "FETCH_SIZE", 9e9), (MARCH, "FETCH_SIZE", 1000.0), (MARCH, "FETCH_SIZE", 1000.0),
               (COPY, "FETCH_SIZE", 5.0)])
    _counters(str(d / "write" / "o_counter_collection.csv"),
              [(MARCH, "WRITE_SIZE", 10.0), (MARCH, "WRITE_SIZE", 30.0), (MARCH, "WRITE_SIZE", 20.0)])
    tf = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tf))
    bench.ingest_traffic(str(d), "w")
    rec = json.load(open(tf))["w"]
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    assert rec["fetch_bytes"] == 1000 * 1024 * 2 and rec["write_bytes"] == 20 * 1024
    assert rec["bytes_per_launch"] == rec["fetch_bytes"] + rec["write_bytes"]
    assert rec["kernel_hash"] == bench.kernel_hash()
    assert bench.load_traffic("w") == rec["bytes_per_launch"]
    # a record taken on other kernel sources is not used
    rec["kernel_hash"] = "0" * 16
    json.dump({"w": rec}, open(tf, "w"))
    assert bench.load_traffic("w") is None
    assert bench.load_traffic("missing") is None


def test_ingest_traffic_without_marcher_records_fails(tmp_path, monkeypatch):
    d = tmp_path / "prof"
    for sub, c in (("copy_fetch", "FETCH_SIZE"), ("copy_write", "WRITE_SIZE"), ("fetch", "FETCH_SIZE"),
                   ("write", "WRITE_SIZE")):
        _counters(str(d / sub / "x_counter_collection.csv"), [(COPY, c, 1024.0)])
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "t.json"))
    with pytest.raises(SystemExit):
        bench.ingest_traffic(str(d), "w")
    assert not (tmp_path / "t.json").exists()


def test_percentile_interpolates():
    assert bench.percentile([], 50) is None
    assert bench.percentile([3.0], 99) == 3.0
    assert bench.percentile([4.0, 1.0, 3.0, 2.0], 50) == 2.5
    assert bench.percentile(list(range(101)), 99) == 99.0


def test_limiter_names_the_timed_kernel():
    assert bench._limiter("graph", "u12").startswith("VALU issue")
    assert bench._limiter("plain", "u12").startswith("the longest ray")
    for form, st in (("graph", "u12"), ("plain", "u16"), ("skip", "u15")):
        note = bench._limiter(form, st)
        assert note.count("(") == note.count(")")
        if "see " in note:
            assert os.path.exists(os.path.join(ROOT, note.split("see ")[1].rstrip(")")))
