"""bench.py's output line on the GPU: the fields and their consistency (one
short run at a pinned launch shape, with the oracle's CPU baseline)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_orbit_line_fields_and_consistency():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "3", "--warmup", "1",
                        "--shape", "4x16x12", "--cpu-budget", "2"], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    line = json.loads(r.stdout.strip().splitlines()[-1])
    for k, v in (("n_gpus", 1), ("steps", 3), ("warmup", 1), ("higher_is_better", True), ("scaling", "weak"),
                 ("vs_baseline", None), ("data", "synthetic"), ("unit", "Gsamples/s")):
        assert line[k] == v, k
    assert line["config"]["workload"] == "brain-orbit-36x512x512-u12-quads" and line["config"]["storage"] == "u12"
    assert line["config"]["layout"] == "quads"
    assert line["config"]["tile"] == [4, 16] and line["config"]["waves_per_block"] == 12
    samples, ms = line["samples_per_step"], line["ms_per_step"]
    assert samples > 0 and ms > 0
    assert abs(line["value"] - samples / (ms * 1e-3) / 1e9) <= 1e-3 * line["value"] + 1e-3
    assert abs(line["fps"] - 36 / (ms * 1e-3)) <= 1e-3 * line["fps"] + 0.1
    rf = line["roofline"]
    # the binding resource: VALU issue, a true ceiling
    assert rf["bound"] == "alu" and rf["unit"] == "T VALU lane-ops/s"
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert abs(rf["peak"] - cus * 4 * 32 * 2.4 / 1e3) <= 1e-3
    assert rf["samples_per_launch"] == samples
    assert 40.0 <= rf["valu_per_sample"] <= 90.0
    if rf.get("counters"):
        # the issued count: SQ_INSTS_VALU x 64 lanes per composited sample
        assert abs(rf["valu_per_sample"] - rf["counters"]["sq_insts_valu"] * 64.0 / samples) <= 1e-3
    lp = rf["loop"]
    assert lp is not None and 0.0 < lp["valu_per_transparent_sample"] < lp["valu_per_compositing_sample"]
    assert abs(rf["achieved"] - samples * rf["valu_per_sample"] / (ms * 1e-3) / 1e12) <= 1e-3 * rf["achieved"] + 1e-3
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) <= 1e-3
    assert 0.0 < rf["frac"] <= 1.0
    lg = rf["logical_gather"]
    assert lg["bytes_per_launch"] == samples * 16 + 36 * 512 * 512 * 16
    assert abs(lg["GB_per_s"] - lg["bytes_per_launch"] / (ms * 1e-3) / 1e9) <= 0.1 + 1e-3 * lg["GB_per_s"]
    assert rf["traffic"] is None or (rf["traffic"] > 0 and 0.0 < rf["fabric"]["frac_of_hbm_peak"] <= 1.0)
    if rf.get("counters"):
        c = rf["counters"]
        assert 0.0 < c["issue_frac_of_busy_cycles"] <= 1.0 and 0.0 < c["lane_utilisation"] <= 1.0
    cb = line["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["unit"] == "Gsamples/s" and cb["value"] > 0 and cb["cores"] >= 1
    assert cb["sample"] and cb["cpu_model"] and cb["nproc"] >= 1
    sk = line["skip_empty"]
    assert sk["images_bitwise_equal"] is True and sk["ms_per_step"] > 0
    sc = line["small_config"]
    assert sc["samples"] == sc["oracle_samples"] > 0
