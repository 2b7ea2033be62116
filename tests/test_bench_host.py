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

MARCH = "void rtv::(anonymous namespace)::march_batch_kernel<6, 4>(char*, rtv::LaunchShape, int, int)"
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
    assert bench._limiter("graph", "u12").startswith("VALU instruction issue")
    assert "see profiles/march_batch_u12_quads_brain_orbit.md" in bench._limiter("graph", "u12", "quads")
    assert bench._limiter("plain", "u12").startswith("the longest ray")
    for form, st, lay in (("graph", "u12", "quads"), ("plain", "u16", "quads"), ("skip", "u15", "cells"),
                          ("graph", "u12", "cells")):
        note = bench._limiter(form, st, lay)
        assert note.count("(") == note.count(")")
        if "see " in note:
            assert os.path.exists(os.path.join(ROOT, note.split("see ")[1].rstrip(")")))


def test_ingest_valu_issue_figures(tmp_path, monkeypatch):
    """Raw counters to issue fractions: 64 lane-operations per wave64 VALU
    instruction against 32 per SIMD per cycle on each of 4 SIMDs per CU, busy
    cycles summed over the 8 XCDs."""
    d = tmp_path / "prof" / "valu"
    os.makedirs(d)
    rows = []
    for disp, scale in ((0, 1.0), (1, 1.0), (2, 3.0)):   # the third dispatch an outlier: medians are taken
        for c, v in (("SQ_INSTS_VALU", 1.0e9 * scale), ("GRBM_GUI_ACTIVE", 8 * 5.0e6 * scale),
                     ("SQ_THREAD_CYCLES_VALU", 57.6e9 * scale), ("SQ_ACTIVE_INST_VALU", 1.0e9 * scale)):
            rows.append({"Dispatch_Id": disp, "Kernel_Name": MARCH, "Counter_Name": c, "Counter_Value": v,
                         "Start_Timestamp": 0, "End_Timestamp": int(2.0e6 * scale)})
    with open(d / "x_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)
    vf = tmp_path / "valu.json"
    monkeypatch.setattr(bench, "VALU_FILE", str(vf))
    bench.ingest_valu(str(tmp_path / "prof"), "w", samples=5.0e10)
    rec = bench.load_valu("w")
    assert rec is not None and rec["kernel_hash"] == bench.kernel_hash()
    assert rec["issue_frac_of_busy_cycles"] == pytest.approx(1.0e9 * 2 / (1024 * 5.0e6))
    assert rec["clock_GHz"] == pytest.approx(2.5)
    assert rec["issue_frac_at_peak_clock"] == pytest.approx(1.0e9 * 2 / (1024 * 2.4 * 2.0e6))
    assert rec["lane_utilisation"] == pytest.approx(0.9)
    assert rec["valu_wave_insts_per_sample"] == pytest.approx(0.02)
    rec["kernel_hash"] = "0" * 16
    json.dump({"w": rec}, open(vf, "w"))
    assert bench.load_valu("w") is None


def test_valu_roofline_is_a_ceiling():
    peak = bench.valu_peak_tops(256)
    assert peak == pytest.approx(256 * 4 * 32 * 2.4 / 1e3)
    r = bench.valu_roofline(1.0e9, 2.0, 50.0, 256)
    assert r["bound"] == "alu" and r["achieved"] == pytest.approx(25.0, abs=1e-3)
    assert r["frac"] == pytest.approx(25.0 / peak, abs=1e-4) and r["frac"] <= 1.0


def test_isa_loop_counts_from_the_built_library():
    """The compositing loop of the batched kernel is found in the built code
    object: per sample one cell load, one paired opacity read and two colour
    reads from LDS; the colour block the wave's vote skips is counted apart.
    The single-view kernel's ring loop is found too."""
    import paper_1211_5595_amd as rt
    from paper_1211_5595_amd import isa
    if not os.path.exists(rt.LIB_PATH):
        pytest.skip("library not built")
    for kind in (rt.U12, rt.U16):
        for layout in (rt.LAYOUT_CELLS, rt.LAYOUT_QUADS):
            lp = isa.loop_profile(rt.LIB_PATH, kind, layout)
            assert lp is not None and lp["lds_per_sample"] == 3.0 and lp["vmem_per_sample"] == 1.0
            assert 30.0 <= lp["valu_per_sample"] <= 90.0
            # three colour lerps, the product T a, three colour FMAs and the transmittance FMA
            assert 8.0 <= lp["valu_per_sample"] - lp["valu_per_transparent_sample"] <= 16.0
    assert isa.loop_profile(rt.LIB_PATH, rt.U12, rt.LAYOUT_CELLS)["valu_per_sample"] < \
        isa.loop_profile(rt.LIB_PATH, rt.U16, rt.LAYOUT_CELLS)["valu_per_sample"]
    # the single-view ring composites without the vote: both entries read whole
    plain = isa.loop_profile(rt.LIB_PATH, rt.U12, rt.LAYOUT_QUADS, "march_plain_kernel")
    assert plain is not None and plain["vmem_per_sample"] == 1.0 and plain["lds_per_sample"] == 2.0
    assert plain["valu_per_transparent_sample"] == plain["valu_per_sample"]


def test_serve_breakdown_splits_latency():
    """Per-request stamps -> submit, queue and service parts; batches in flight
    at each launch and requests waiting at each arrival."""
    recs = []
    # three batches: A (2 requests) 0..1 ms, B (1) 0.5..2 ms overlapping A, C (1) 5..6 ms
    for k, (tgt, ts, tl, td, b) in enumerate([(0.0, 0.0, 0.0001, 0.001, 2), (0.0, 0.00005, 0.0001, 0.001, 2),
                                             (0.0002, 0.0002, 0.0005, 0.002, 1), (0.005, 0.005, 0.005, 0.006, 1)]):
        recs.append({"target": tgt, "t_submit": ts, "t_launch": tl, "t_done": td, "batch": b, "side": 256 + 64 * k})
    bd = bench.serve_breakdown(recs)
    assert bd["batches"] == 3
    assert bd["batch_size_hist"] == {"1": 2, "2": 1}
    assert bd["batches_in_flight_at_launch_hist"] == {"0": 2, "1": 1}
    assert bd["requests_waiting_at_arrival_max"] == 1
    # the slowest request (1.8 ms, arrived at 0.2 ms) waited 0.3 ms and rendered 1.5 ms
    s = bd["slowest_1pct_median"]
    assert s["n"] == 1 and abs(s["queue_ms"] - 0.3) < 1e-9 and abs(s["service_ms"] - 1.5) < 1e-9
    assert bench.serve_breakdown([]) is None
