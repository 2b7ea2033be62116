"""Benchmark: ray samples per second and frames per second of the raycaster.

Default workload (one "step"): the 36-view orbit of the seeded 256x256x160
uint16 brain phantom (spacing 0.9x0.9x1.2 mm), 512x512 perspective images,
step 0.5 voxel, 4096-entry RGBA transfer function, early termination at
0.99.  Volume and transfer function are resident in HBM before timing; a
step renders all 36 views in one persistent batched launch.  The plain
per-view launch is timed beside it, and single-view latencies give p50/p99.

Samples are counted by the kernels' own counter in an untimed pass (the
count is deterministic and equals the FP64 oracle's except on tie pixels).

Output: one JSON line (see the fields below).  Only one GPU is used.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# Vector-ALU peak: MI355X's fp32 vector rate, 157.3 TFLOP/s, counts a fused
# multiply-add as two flops, i.e. 78.6 T lane-operations per second: 256 CUs x
# 4 SIMDs x 32 lanes per cycle x 2.4 GHz (a wave64 instruction every 2 cycles
# per SIMD; independent VALU instructions of two waves can issue together).
# Every VALU instruction counts as one lane-operation per lane, whatever its
# own rate (conversions, 24-bit multiplies and mixed-precision FMAs issue at
# half that rate, 64-bit adds slower still).
CLOCK_GHZ = 2.4
SIMDS_PER_CU = 4
LANE_OPS_PER_SIMD_CYCLE = 32
N_XCC = 8
KERNEL_SOURCES = ["paper_1211_5595_amd/csrc/march.hip", "paper_1211_5595_amd/csrc/ff_math.h",
                  "paper_1211_5595_amd/csrc/rt_internal.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
VALU_FILE = os.path.join(ROOT, "profiles", "valu_counters.json")


def valu_peak_tops(cus: int = 256) -> float:
    """VALU peak in T lane-operations per second (the fp32 vector rate)."""
    return cus * SIMDS_PER_CU * LANE_OPS_PER_SIMD_CYCLE * CLOCK_GHZ / 1e3


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(workload: str):
    """HBM bytes per launch measured with rocprofv3 counters, if they were
    taken on the current kernel sources."""
    try:
        data = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    rec = data.get(workload)
    if not rec or rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


def _counter_per_dispatch(csv_path, kernel_prefix, counter):
    """Median per-dispatch value of `counter` over the dispatches of the
    kernels whose name starts with kernel_prefix (rocprofv3 counter CSV)."""
    import csv
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(csv_path))
            if r["Counter_Name"] == counter and r["Kernel_Name"].startswith(kernel_prefix)]
    if not vals:
        raise SystemExit(f"no {counter} records for {kernel_prefix} in {csv_path}")
    vals.sort()
    return vals[len(vals) // 2]


def ingest_traffic(d, key, copy_bytes=1 << 30):
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the marcher, each
    scaled by what the counter reads for a plain copy of copy_bytes (the
    --probe-copy kernel), recorded with the kernel source hash."""
    import glob
    one = lambda sub: glob.glob(os.path.join(d, sub, "*counter_collection.csv"))[0]
    copy_k = "__amd_rocclr_copyBuffer"
    march_k = "void rtv::(anonymous namespace)::march_batch_kernel<"
    fetch_scale = copy_bytes / (_counter_per_dispatch(one("copy_fetch"), copy_k, "FETCH_SIZE") * 1024.0)
    write_scale = copy_bytes / (_counter_per_dispatch(one("copy_write"), copy_k, "WRITE_SIZE") * 1024.0)
    fetch = _counter_per_dispatch(one("fetch"), march_k, "FETCH_SIZE") * 1024.0 * fetch_scale
    write = _counter_per_dispatch(one("write"), march_k, "WRITE_SIZE") * 1024.0 * write_scale
    try:
        data = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        data = {}
    data[key] = {"kernel_hash": kernel_hash(), "bytes_per_launch": int(round(fetch + write)),
                 "fetch_bytes": int(round(fetch)), "write_bytes": int(round(write)),
                 "fetch_scale": fetch_scale, "write_scale": write_scale}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    print(json.dumps({key: data[key]}))


def load_valu(workload: str):
    """VALU counters per launch of the timed kernel (rocprofv3), if they were
    taken on the current kernel sources."""
    try:
        data = json.load(open(VALU_FILE))
    except (OSError, ValueError):
        return None
    rec = data.get(workload)
    if not rec or rec.get("kernel_hash") != kernel_hash():
        return None
    return rec


def ingest_valu(d, key, samples, cus=256, kernel="march_batch_kernel<6, 4>"):
    """Raw SQ/GRBM counters of the marcher (medians per dispatch of one
    rocprofv3 --pmc pass, CSVs under DIR/valu) turned into issue figures:
    SQ_INSTS_VALU wave instructions x 64 lanes against the VALU peak of 32
    lane-operations per SIMD per cycle, over the cycles the GPU was busy
    (GRBM_GUI_ACTIVE, summed over the XCDs) and over the dispatch time at the
    2.4 GHz peak clock; lane utilisation SQ_THREAD_CYCLES_VALU / (64
    SQ_ACTIVE_INST_VALU).  `samples` is the composited-sample count of one
    launch (bench.py's counting pass)."""
    import csv
    import glob
    path = glob.glob(os.path.join(d, "valu", "*counter_collection.csv"))[0]
    march_k = "void rtv::(anonymous namespace)::" + kernel
    med = lambda c: _counter_per_dispatch(path, march_k, c)
    insts = med("SQ_INSTS_VALU")
    gui = med("GRBM_GUI_ACTIVE") / N_XCC
    thread = med("SQ_THREAD_CYCLES_VALU")
    active = med("SQ_ACTIVE_INST_VALU")
    durs = sorted(float(r["End_Timestamp"]) - float(r["Start_Timestamp"]) for r in csv.DictReader(open(path))
                  if r["Kernel_Name"].startswith(march_k) and r["Counter_Name"] == "SQ_INSTS_VALU"
                  and r.get("End_Timestamp"))
    ns = durs[len(durs) // 2] if durs else None
    simds = cus * SIMDS_PER_CU
    rec = {"kernel_hash": kernel_hash(), "sq_insts_valu": insts, "grbm_gui_active_cycles": gui,
           "sq_thread_cycles_valu": thread, "sq_active_inst_valu": active, "samples_per_launch": int(samples),
           "valu_wave_insts_per_sample": insts / samples,
           "lane_utilisation": thread / (64.0 * active) if active else None,
           "issue_frac_of_busy_cycles": insts * 64.0 / (simds * LANE_OPS_PER_SIMD_CYCLE * gui) if gui else None}
    if ns:
        rec["dispatch_ns"] = ns
        rec["clock_GHz"] = gui / ns if gui else None
        rec["issue_frac_at_peak_clock"] = insts * 64.0 / (simds * LANE_OPS_PER_SIMD_CYCLE * CLOCK_GHZ * ns)
    try:
        data = json.load(open(VALU_FILE))
    except (OSError, ValueError):
        data = {}
    data[key] = rec
    with open(VALU_FILE, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    print(json.dumps({key: rec}))


def valu_roofline(samples, ms_per_launch, valu_per_sample, cus):
    """Vector-ALU roofline of one launch: the VALU lane-slots the launch
    issues (samples x VALU wave instructions per sample x 64 lanes / 64
    samples per wave, i.e. samples x `valu_per_sample`) per second, against
    the fp32 vector issue peak in lane-operations."""
    peak = valu_peak_tops(cus)
    achieved = samples * valu_per_sample / (ms_per_launch * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3), "unit": "T VALU lane-ops/s",
            "frac": round(achieved / peak, 4)}


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * p / 100.0
    f = int(k)
    c = min(f + 1, len(xs) - 1)
    return xs[f] + (xs[c] - xs[f]) * (k - f)


def cpu_baseline(vol_np, tf_np, cams, spacing, width, height, step, cutoff, vmax, budget_s=20.0):
    """The FP64 oracle as it stands, all host threads, on whole views of the
    same workload until about budget_s seconds have passed."""
    import oracle
    V = oracle.Volume(vol_np, spacing)
    T = oracle.TF(tf_np, 0.0, vmax)
    n_views, samples = 0, 0
    t0 = time.perf_counter()
    for cam in cams:
        r = oracle.render(V, T, cam, width, height, step, cutoff)
        samples += int(r.counts.sum())
        n_views += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    # one core, on the first view alone
    t1 = time.perf_counter()
    r1 = oracle.render(V, T, cams[0], width, height, step, cutoff, nthreads=1)
    dt1 = time.perf_counter() - t1
    return {"value": samples / dt / 1e9, "unit": "Gsamples/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"{n_views} of the {len(cams)} orbit views, {width}x{height}, whole images",
            "fps": n_views / dt, "seconds": dt, **_lscpu(),
            "single_core": {"value": int(r1.counts.sum()) / dt1 / 1e9, "unit": "Gsamples/s", "cores": 1,
                            "sample": "orbit view 0, whole image", "seconds": dt1}}


def small_config(reps=200):
    """The small correctness workload (the 64x64x32 8-bit phantom, one
    orthographic 128x128 view, step 0.5, cutoff 0.99): the GPU's single-view
    time (HIP events around each launch, p50 over reps) and the oracle's on
    the same view, all host threads."""
    import torch

    import oracle
    import paper_1211_5595_amd as rt
    import workloads as W

    cfg = W.CONFIG_SMALL
    vs, ts = cfg["volume"], cfg["tf"]
    width, height, step, cutoff = cfg["width"], cfg["height"], cfg["step_vox"], cfg["cutoff"]
    v = W.phantom_small(vs.seed, dims=vs.dims, spacing=vs.spacing)
    t = W.random_tf(ts.K, ts.seed, alpha_max=ts.alpha_max)
    cam = W.ortho_camera_small(vs.dims, vs.spacing)
    vol = rt.Volume(v, vs.spacing, storage=rt.U8)
    tf = rt.TransferFunction(t, ts.vmin, ts.vmax)
    counter = torch.zeros(1, dtype=torch.int64, device="cuda")
    out = rt.render(vol, tf, cam, width, height, step, cutoff, sample_counter=counter)
    torch.cuda.synchronize()
    samples = int(counter.item())
    stream = torch.cuda.current_stream()
    lat = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        rt.render(vol, tf, cam, width, height, step, cutoff, out=out)
        e1.record(stream)
        e1.synchronize()
        lat.append(e0.elapsed_time(e1))
    p50 = percentile(lat, 50)
    V, T = oracle.Volume(v, vs.spacing), oracle.TF(t, ts.vmin, ts.vmax)
    t0 = time.perf_counter()
    r = oracle.render(V, T, cam, width, height, step, cutoff)
    dt = time.perf_counter() - t0
    return {"workload": "small-64x64x32-u8-ortho-128x128", "samples": samples,
            "gpu_p50_ms": p50, "gpu_gsamples_per_s": round(samples / (p50 * 1e-3) / 1e9, 3),
            "cpu_oracle_ms": round(dt * 1e3, 3), "cpu_gsamples_per_s": round(int(r.counts.sum()) / dt / 1e9, 4),
            "cpu_cores": oracle.max_threads(), "oracle_samples": int(r.counts.sum())}


def _lscpu() -> dict:
    """CPU model and processor count as lscpu and nproc report them."""
    import subprocess
    out = {"cpu_model": "unknown", "lscpu_cpus": None, "nproc": None}
    try:
        r = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10)
        for line in r.stdout.splitlines():
            k, _, v = line.partition(":")
            if k.strip() == "Model name":
                out["cpu_model"] = v.strip()
            elif k.strip() == "CPU(s)":
                out["lscpu_cpus"] = int(v.strip())
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    try:
        r = subprocess.run(["nproc"], capture_output=True, text=True, timeout=10)
        out["nproc"] = int(r.stdout.strip())
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    return out


def _cpu_model() -> str:
    return _lscpu()["cpu_model"]


def probe_copy(gib: float = 1.0, reps: int = 10, quiet: bool = False):
    """Plain device copy of a known size (for counter calibration and the
    achievable-bandwidth figure); returns the copy's read+write GB/s."""
    import torch
    n = int(gib * (1 << 30))
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    if not quiet:
        print(json.dumps({"probe": "copy", "bytes_read": n, "bytes_written": n, "ms": ms,
                          "GB_per_s": 2 * n / ms / 1e6}))
    return 2 * n / ms / 1e6


def _timed(fn, steps, warmup):
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _limiter(form, storage, layout="quads"):
    """What bounds the timed kernel, with the profile summary that shows it."""
    if form in ("batch", "graph"):
        # the caches serve three quarters of the logical gathers, so their rate
        # can exceed the HBM peak; what binds is vector-instruction issue
        text, prof = "VALU instruction issue (raw SQ_INSTS_VALU over busy cycles", \
            f"profiles/march_batch_{storage}_{layout}_brain_orbit.md"
    elif form == "skip":
        text, prof = "VALU instruction issue of the samples taken (skipped ones cost a leap per brick", \
            "profiles/march_batch_other_forms_brain_orbit.md"
    else:
        # one launch per view: the longest ray's own instruction stream
        text, prof = "the longest ray of each lone view (one launch per view", \
            "profiles/march_batch_other_forms_brain_orbit.md"
    here = os.path.dirname(os.path.abspath(__file__))
    return text + (f", see {prof})" if os.path.exists(os.path.join(here, prof)) else ")")


def _count(rt, jobs):
    import torch
    counter = torch.zeros(1, dtype=torch.int64, device="cuda")
    rt.render_batch(jobs, sample_counter=counter)
    torch.cuda.synchronize()
    return int(counter.item())


def _plain_caller(rt, jobs):
    """The plain per-view launches with their ctypes arguments built once, so
    the timed loop is one C call per view."""
    import ctypes as C
    L = rt.lib()
    stream = rt._stream_ptr()
    calls = []
    for j in jobs:
        dims = (C.c_int64 * 3)(*j.volume.dims)
        bg = (C.c_float * 4)(*[float(x) for x in j.bg])
        calls.append((C.c_void_p(j.volume.handle), dims, None, C.c_void_p(j.tf.handle),
                      C.byref(rt.make_camera(j.camera)), j.width, j.height, C.c_double(j.step_vox),
                      C.c_double(j.alpha_cutoff), bg, C.c_void_p(j.out.data_ptr()), None, stream))

    def run():
        for c in calls:
            if L.rt_render(*c) != 0:
                raise RuntimeError(L.rt_last_error().decode())
    return run


def _storage(rt, args):
    """Device storage of the 12-bit uint16 phantoms (every choice holds them exactly)."""
    return {"u16": rt.U16, "u15": rt.U15, "u12": rt.U12}[args.storage]


def _layout(rt, args):
    return {"cells": rt.LAYOUT_CELLS, "poly": rt.LAYOUT_POLY, "linear": rt.LAYOUT_LINEAR,
            "quads": rt.LAYOUT_QUADS}[args.layout]


def _contract(metric, value, unit, args, ms_step, dtype, config, **extra):
    line = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}
    line.update(extra)
    return line


def bench_precision(args):
    """The 256x256x160 phantom stored as u16 (reference), f16 and per-brick
    scaled 8-bit codes (B=16); 8 orbit views at 1024x1024, step 0.25 voxel.
    Per storage type: throughput, algorithmic GB/s, and the two-part error
    against the FP64 oracle on two of the views: arithmetic (GPU vs oracle on
    the stored field, tie-aware) and storage (oracle on the stored field vs
    oracle on the u16 original)."""
    import numpy as np
    import torch

    import oracle
    import paper_1211_5595_amd as rt
    import workloads as W

    cfg = W.CONFIG_BRAIN
    vs, ts = cfg["volume"], cfg["tf"]
    size, step, cutoff, n_views = 1024, 0.25, cfg["cutoff"], 8
    vol_np = W.phantom_brain(vs.seed, dims=vs.dims, spacing=vs.spacing)
    tf_np = W.random_tf(ts.K, ts.seed, alpha_max=ts.alpha_max)
    cams = W.orbit_cameras(vs.dims, vs.spacing, n_views)
    torch.cuda.set_device(0)
    tf = rt.TransferFunction(tf_np, ts.vmin, ts.vmax)
    otf = oracle.TF(tf_np, ts.vmin, ts.vmax)
    err_views = [0, 3]
    cpu = None
    ref_u16 = {}
    results = {}
    for name, storage, brick, elem_bytes in [("u16", rt.U16, 0, 2), ("u12", rt.U12, 0, 2), ("f16", rt.F16, 0, 2),
                                             ("u8_brick16", rt.U8_BRICKSCALED, 16, 1)]:
        vol = rt.Volume(vol_np, vs.spacing, storage=storage, brick=brick)
        outs = [torch.empty((size, size, 4), dtype=torch.float32, device="cuda") for _ in range(n_views)]
        jobs = [rt.Job(vol, tf, cam, size, size, step, cutoff, out=o) for cam, o in zip(cams, outs)]
        plan = rt.BatchPlan(n_views, storage)
        samples = _count(rt, jobs)
        ms = _timed(lambda: plan.launch(jobs), args.steps, args.warmup)
        algo = samples * 8 * elem_bytes + n_views * size * size * 16
        if name in ("u16", "u12"):  # both hold the 12-bit grid exactly
            ofield = oracle.Volume(vol_np, vs.spacing)
        elif name == "f16":
            ofield = oracle.Volume(vol_np.astype(np.float16).astype(np.float64), vs.spacing)
        else:
            ofield = oracle.Volume.from_u8_bricks(vol_np, vs.spacing, 16)
        plan.launch(jobs)
        torch.cuda.synchronize()
        if name == "u16":  # the oracle's own time on one whole view of this workload, all host threads
            t0 = time.perf_counter()
            r0 = oracle.render(ofield, otf, cams[0], size, size, step, cutoff)
            dt0 = time.perf_counter() - t0
            cpu = {"value": round(int(r0.counts.sum()) / dt0 / 1e9, 4), "unit": "Gsamples/s",
                   "cores": oracle.max_threads(), "kind": "oracle", "seconds": round(dt0, 3),
                   "sample": f"view 0, whole {size}x{size} image, 16-bit field"}
        arith_max, arith_sum, stor_max, stor_sum, npx = 0.0, 0.0, 0.0, 0.0, 0
        for vi in err_views:
            got = outs[vi].cpu().numpy().astype(np.float64)
            r = oracle.render(ofield, otf, cams[vi], size, size, step, cutoff, tie_delta=1e-6, want_band=True)
            dist = np.maximum(np.maximum(r.band_lo - got, got - r.band_hi), 0.0)
            arith_max = max(arith_max, float(dist.max()))
            arith_sum += float(np.abs(got - r.image).sum())
            if name == "u16":
                ref_u16[vi] = r.image
            stor = np.abs(r.image - ref_u16[vi])
            stor_max = max(stor_max, float(stor.max()))
            stor_sum += float(stor.sum())
            npx += got.size
        results[name] = {
            "gsamples_per_s": round(samples / (ms * 1e-3) / 1e9, 3), "fps": round(n_views / (ms * 1e-3), 1),
            "ms_per_launch": round(ms, 4), "samples_per_launch": samples,
            "algorithmic_GB_per_s": round(algo / (ms * 1e-3) / 1e9, 1),
            "volume_bytes": vol.nbytes,
            "error_vs_fp64_oracle": {"arithmetic_max": arith_max, "arithmetic_mean": arith_sum / npx,
                                     "storage_max": stor_max, "storage_mean": stor_sum / npx,
                                     "views_checked": err_views}}
        del plan, vol
    line = _contract("ray samples/sec (G/s) per storage type at 1024x1024 over 256x256x160, step 0.25; "
                     "max/mean RGBA error vs FP64 oracle", results["u16"]["gsamples_per_s"], "Gsamples/s", args,
                     results["u16"]["ms_per_launch"], "f32",
                     {"workload": "brain-precision-8x1024x1024-step0.25", "volume": list(vs.dims),
                      "views": n_views, "image": [size, size], "step_vox": step, "alpha_cutoff": cutoff,
                      "tf_entries": ts.K, "storage": ["u16", "u12", "f16", "u8_brick16"], "launch": "graph"},
                     by_storage=results, cpu_baseline=cpu)
    print(json.dumps(line), flush=True)


def bench_projection(args):
    """Every ray function over the 36 orbit views of the 256x256x160 u16
    phantom at 512x512, step 0.5, one graph-captured persistent launch per
    step: compositing, maximum-intensity, X-ray and average-intensity
    projection (every lattice sample, no early termination), thresholding to
    the window [1200, 2600] (with and without empty-space skipping) and the
    iso-surface at 1000 (samples up to the first hit)."""
    import torch

    import paper_1211_5595_amd as rt
    import workloads as W

    cfg = W.CONFIG_BRAIN
    vs, ts = cfg["volume"], cfg["tf"]
    width, height, step, n_views = cfg["width"], cfg["height"], cfg["step_vox"], cfg["n_views"]
    vol_np = W.phantom_brain(vs.seed, dims=vs.dims, spacing=vs.spacing)
    cams = W.orbit_cameras(vs.dims, vs.spacing, n_views)
    torch.cuda.set_device(0)
    st, lay = _storage(rt, args), _layout(rt, args)
    vol = rt.Volume(vol_np, vs.spacing, storage=st, layout=lay)
    tf_np = W.random_tf(ts.K, ts.seed, alpha_max=ts.alpha_max)
    results = {}
    plan = rt.BatchPlan(n_views, st, layout=lay)
    plan_s = rt.BatchPlan(n_views, st, layout=lay, skip_empty=True)
    for name, fn, top, lo, hi, skip in [("composite", rt.COMPOSITE, ts.vmax, 0.0, 0.0, False),
                                        ("mip", rt.MIP, ts.vmax, 0.0, 0.0, False),
                                        ("xray", rt.XRAY, ts.vmax * 150.0, 0.0, 0.0, False),
                                        ("average", rt.AVERAGE, ts.vmax, 0.0, 0.0, False),
                                        ("threshold", rt.THRESHOLD, ts.vmax, 1200.0, 2600.0, False),
                                        ("threshold_skip", rt.THRESHOLD, ts.vmax, 1200.0, 2600.0, True),
                                        ("iso", rt.ISO, ts.vmax, 1000.0, 0.0, False)]:
        tf = rt.TransferFunction(tf_np, ts.vmin, top)
        outs = [torch.empty((height, width, 4), dtype=torch.float32, device="cuda") for _ in range(n_views)]
        jobs = [rt.Job(vol, tf, cam, width, height, step, cfg["cutoff"], out=o, ray_function=fn, iso_value=lo,
                       iso_high=hi, skip_empty=skip) for cam, o in zip(cams, outs)]
        samples = _count(rt, jobs)
        pl = plan_s if skip else plan
        ms = _timed(lambda: pl.launch(jobs), args.steps, args.warmup)
        results[name] = {"gsamples_per_s": round(samples / (ms * 1e-3) / 1e9, 3),
                         "fps": round(n_views / (ms * 1e-3), 1), "ms_per_launch": round(ms, 4),
                         "samples_per_launch": samples,
                         # skipped samples are counted but never gathered: no byte rate for them
                         "algorithmic_GB_per_s": None if skip else
                         round((samples * 16 + n_views * width * height * 16) / (ms * 1e-3) / 1e9, 1)}
    line = _contract("ray samples/sec (G/s) + fps per ray function at 512x512 over 256x256x160",
                     results["mip"]["gsamples_per_s"], "Gsamples/s", args, results["mip"]["ms_per_launch"], "f32",
                     {"workload": f"brain-ray-functions-36x512x512-{args.storage}-{args.layout}",
                      "volume": list(vs.dims), "views": n_views, "storage": args.storage, "layout": args.layout,
                      "image": [width, height], "step_vox": step, "tf_entries": ts.K,
                      "ray_functions": list(results), "launch": "graph"},
                     by_ray_function=results)
    print(json.dumps(line), flush=True)


def bench_batch(args):
    """32 seeded phantoms of uneven sizes (u16), 4 random views each at
    256..1024 square, one transfer function per phantom: one persistent
    graph-captured launch against 128 plain per-view launches."""
    import torch

    import paper_1211_5595_amd as rt
    import workloads as W

    torch.cuda.set_device(0)
    specs, views = W.random_views(seed=4)
    t0 = time.perf_counter()
    vols, tfs = [], []
    for i, sp in enumerate(specs):
        v = W.phantom_brain(sp.seed, dims=sp.dims, spacing=sp.spacing)
        vols.append(rt.Volume(v, sp.spacing, storage=_storage(rt, args), layout=_layout(rt, args)))
        tfs.append(rt.TransferFunction(W.random_tf(4096, 1000 + i, alpha_max=0.05), 0.0, 4095.0))
        print(f"volume {i} {sp.dims} ready", file=sys.stderr, flush=True)
    gen_s = time.perf_counter() - t0
    jobs = [rt.Job(vols[vi], tfs[vi], cam, side, side, 0.5, 0.99) for vi, cam, side in views]
    jobs_s = [rt.Job(vols[vi], tfs[vi], cam, side, side, 0.5, 0.99, skip_empty=True) for vi, cam, side in views]
    tuned = tuned_s = None
    shape, shape_s = {}, {}
    if not args.no_autotune:  # ray-tile shape and workgroup size of each launch form, timed on this batch
        from paper_1211_5595_amd import autotune
        tuned = autotune.tune_batch(jobs, _storage(rt, args), _layout(rt, args))
        tuned_s = autotune.tune_batch(jobs_s, _storage(rt, args), _layout(rt, args), skip_empty=True)
        shape = dict(tile=tuple(tuned["tile"]), waves_per_block=tuned["waves_per_block"])
        shape_s = dict(tile=tuple(tuned_s["tile"]), waves_per_block=tuned_s["waves_per_block"])
    plan = rt.BatchPlan(len(jobs), _storage(rt, args), layout=_layout(rt, args), **shape)
    samples = _count(rt, jobs)

    plain = _plain_caller(rt, jobs)
    ms_graph = _timed(lambda: plan.launch(jobs), args.steps, args.warmup)
    ms_plain = _timed(plain, args.steps, args.warmup)
    # the same batch with exact empty-space skipping (same images, fewer samples gathered)
    plan_s = rt.BatchPlan(len(jobs), _storage(rt, args), layout=_layout(rt, args), skip_empty=True, **shape_s)
    ms_skip = _timed(lambda: plan_s.launch(jobs_s), args.steps, args.warmup)
    torch.cuda.synchronize()
    same = all(torch.equal(a.out, b.out) for a, b in zip(jobs, jobs_s))
    pixels = sum(j.width * j.height for j in jobs)
    algo = samples * 16 + pixels * 16
    g = samples / (ms_graph * 1e-3) / 1e9
    # measured counters of this launch (rocprofv3, same kernel sources and launch shape), if taken:
    # fabric bytes and VALU issue against their peaks -- neither is saturated, the launch waits on
    # lines from beyond the caches (the volumes are far larger than the Infinity Cache)
    tile = tuple(shape.get("tile", (8, 8)))
    waves = shape.get("waves_per_block", 12)
    key = f"uneven-batch-32vol-128views-{args.storage}-{args.layout}:graph:{tile[0]}x{tile[1]}x{waves}"
    traffic, cnt = load_traffic(key), load_valu(key)
    sec = ms_graph * 1e-3
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    counters = {
        "key": key,
        "fabric": None if traffic is None else {
            "bytes_per_launch": traffic, "GB_per_s": round(traffic / sec / 1e9, 1),
            "frac_of_hbm_peak": round(traffic / sec / 1e9 / PEAK_HBM_GBS, 4),
            "note": "FETCH_SIZE x 2 + WRITE_SIZE x 1 per launch (scales from a plain copy)"},
        "valu_issue": None if cnt is None else {
            "lane_slots_T_per_s": round(cnt["sq_insts_valu"] * 64.0 / sec / 1e12, 3),
            "frac_of_peak": round(cnt["sq_insts_valu"] * 64.0 / sec / 1e12 / valu_peak_tops(cus), 4),
            "lane_utilisation": cnt.get("lane_utilisation"),
            "issue_frac_of_busy_cycles": cnt.get("issue_frac_of_busy_cycles")},
    }
    line = _contract(f"ray samples/sec (G/s): 128 views of 32 uneven 12-bit volumes stored as {args.storage}, one "
                     "persistent graph launch vs 128 plain launches", round(g, 3), "Gsamples/s", args, ms_graph, "f32",
                     {"workload": f"uneven-batch-32vol-128views-{args.storage}-{args.layout}", "volumes": len(specs),
                      "views": len(jobs), "source_dtype": "u16 (12-bit range)", "storage": args.storage,
                      "layout": args.layout,
                      "sizes": sorted({s.dims for s in specs}), "image_sides": [min(j.width for j in jobs),
                                                                              max(j.width for j in jobs)],
                      "step_vox": 0.5, "alpha_cutoff": 0.99, "tf_entries": 4096, "launch": "graph",
                      "tile": list(shape.get("tile", (8, 8))), "waves_per_block": shape.get("waves_per_block", 12)},
                     autotune={"graph": tuned, "graph_skip_empty": tuned_s},
                     samples_per_step=samples, pixels_per_step=pixels,
                     ms_per_step_by_form={"graph": round(ms_graph, 4), "plain_128_launches": round(ms_plain, 4),
                                          "graph_skip_empty": round(ms_skip, 4)},
                     skip_empty_images_bitwise_equal=bool(same), counters=counters,
                     gsamples_per_s_by_form={"graph": round(g, 3),
                                             "plain_128_launches": round(samples / (ms_plain * 1e-3) / 1e9, 3)},
                     speedup_vs_plain=round(ms_plain / ms_graph, 3),
                     algorithmic_GB_per_s=round(algo / (ms_graph * 1e-3) / 1e9, 1),
                     volume_bytes_total=sum(v.nbytes for v in vols), generation_s=round(gen_s, 1))
    print(json.dumps(line), flush=True)


def serve_breakdown(recs):
    """Where the latency of served requests goes.  recs: one dict per request
    with its arrival `target`, the server's stamps t_submit, t_launch (batch
    launched), t_done (completion seen by the server thread), the size of its
    batch and its image side, all on one monotonic clock.  Returns
    percentiles of the submit delay, queue wait and batch service time, those
    of the slowest 1 % beside those of all requests, the batch sizes, and the
    server's occupancy: batches already in flight when each batch launched
    and requests waiting when each request arrived."""
    import numpy as np
    if not recs:
        return None
    g = lambda k: np.array([r[k] for r in recs], dtype=np.float64)
    target, ts, tl, td = g("target"), g("t_submit"), g("t_launch"), g("t_done")
    bsz, side = g("batch"), g("side")
    lat, sub, que, svc = td - target, ts - target, tl - ts, td - tl
    ms = lambda a, q: round(float(np.percentile(a, q)) * 1e3, 4) if a.size else None
    tail = lat >= np.percentile(lat, 99)
    part = lambda m: {"n": int(m.sum()), "latency_ms": ms(lat[m], 50), "submit_ms": ms(sub[m], 50),
                      "queue_ms": ms(que[m], 50), "service_ms": ms(svc[m], 50),
                      "batch_size": round(float(bsz[m].mean()), 2), "image_side": round(float(side[m].mean()), 1)}
    # one interval per batch (its requests share launch and completion stamps)
    batches = sorted({(a, b) for a, b in zip(tl, td)})
    starts = np.array([b[0] for b in batches])
    ends = np.array([b[1] for b in batches])
    in_flight = np.array([int(((starts < s0) & (ends > s0)).sum()) for s0 in starts])
    waiting = np.array([int(((ts <= t) & (tl > t)).sum()) - 1 for t in ts])
    hist = lambda a: {str(int(k)): int(v) for k, v in zip(*np.unique(a, return_counts=True))}
    return {"p50": {"submit_ms": ms(sub, 50), "queue_ms": ms(que, 50), "service_ms": ms(svc, 50)},
            "p99": {"submit_ms": ms(sub, 99), "queue_ms": ms(que, 99), "service_ms": ms(svc, 99)},
            "all_median": part(np.ones_like(tail)), "slowest_1pct_median": part(tail),
            "batches": len(batches), "batch_size_hist": hist(bsz[np.unique(tl, return_index=True)[1]]),
            "batches_in_flight_at_launch_hist": hist(in_flight),
            "requests_waiting_at_arrival_p50": float(np.percentile(waiting, 50)),
            "requests_waiting_at_arrival_p99": float(np.percentile(waiting, 99)),
            "requests_waiting_at_arrival_max": int(waiting.max())}


def bench_serve(args):
    """Poisson stream (200 req/s, seed 300) over 16 resident 12-bit volumes (4 of
    each batch size, seeds 200+i); each request has its own camera, square
    size in 256..1024 and transfer function.  Served with continuous batching
    under a loose and a tight HBM budget, and serially (one plain render at a
    time, in arrival order) on the same GPU; the first 200 requests are
    warm-up.  A second, 20x faster stream shows saturation."""
    import numpy as np
    import torch

    import paper_1211_5595_amd as rt
    import workloads as W
    from paper_1211_5595_amd.serve import GpuExecutor, NativeServer, RenderRequest, Server

    torch.cuda.set_device(0)
    sp = (0.9, 0.9, 1.2)
    dims = [d for d in W.BATCH_SIZES for _ in range(4)]
    ex = GpuExecutor(n_streams=3, max_batch=64, storage=_storage(rt, args),  # exact empty-space skipping on
                     tile_order=args.tile_order or 2, layout=_layout(rt, args), batch_form=args.batch_form)
    for i, d in enumerate(dims):
        ex.add_volume(i, W.phantom_brain(200 + i, dims=d, spacing=sp), sp)
        print(f"volume {i} {d} resident", file=sys.stderr, flush=True)
    n_req, warm = args.requests, min(200, args.requests // 10)
    trace = W.poisson_requests(300, n_req, rate_hz=200.0, n_volumes=len(dims), volume_dims=dims, spacing=sp)
    reqs = [RenderRequest(r["volume"], r["camera"], r["side"], r["side"],
                          W.random_tf(4096, r["tf_seed"], alpha_max=0.05), 0.0, 4095.0, 0.5, 0.99) for r in trace]

    def wait_until(t):
        while True:
            d = t - time.perf_counter()
            if d <= 0:
                return
            time.sleep(d - 2e-4 if d > 5e-4 else 0)

    def summarize(lat, samples, t_first, t_last, n):
        a = np.array(lat) * 1e3
        span = t_last - t_first
        return {"p50_ms": round(float(np.percentile(a, 50)), 4), "p99_ms": round(float(np.percentile(a, 99)), 4),
                "mean_ms": round(float(a.mean()), 4), "max_ms": round(float(a.max()), 4),
                "requests_per_s": round(n / span, 1), "gsamples_per_s": round(samples / span / 1e9, 3),
                "requests": n}

    def served(budget, speed=1.0, n=None):
        n = n or n_req
        srv = Server(ex, budget, max_batch=64)
        srv.start()
        t0 = time.perf_counter() + 0.05
        futs = []
        for k in range(n):
            target = t0 + trace[k]["t"] / speed
            wait_until(target)
            futs.append((target, srv.submit(reqs[k])))
        srv.stop(drain=True)
        w = warm if speed == 1.0 else 0
        lat = [f.t_done - tgt for tgt, f in futs[w:]]
        samples = sum(f.samples or 0 for _, f in futs[w:])
        for _, f in futs:
            f.result(0)
        out = summarize(lat, samples, futs[w][0], max(f.t_done for _, f in futs[w:]), n - w)
        out.update({"budget_bytes": budget, "peak_bytes": srv.peak_bytes, "batches": srv.batches,
                    "mean_batch": round((n) / max(srv.batches, 1), 2)})
        return out

    def served_native(pool_bytes, speed=1.0, n=None):
        """The same stream through the library's native server (rt_serve.h):
        admission against an image pool, continuous batching, no Python in
        the request loop.  Latency = completion time stamped by the server
        thread (CLOCK_MONOTONIC, the clock of perf_counter) - arrival time."""
        n = n or n_req
        counter = torch.zeros(1, dtype=torch.int64, device="cuda")
        srv = NativeServer(pool_bytes, n_streams=3, max_batch=64, storage=_storage(rt, args),
                           tile_order=args.tile_order or 2, layout=_layout(rt, args), batch_form=args.batch_form,
                           sample_counter=counter)
        srv.volumes = ex.volumes                  # the same resident volumes
        import queue as _q
        import threading as _th
        w = warm if speed == 1.0 else 0
        lat, done, failed, recs = [], [], [], []
        tickets = _q.Queue()

        def consume():  # the client side: take each image as it completes and give its memory back
            i = 0
            while True:
                item = tickets.get()
                if item is None:
                    return
                target, t, side = item
                info = srv.wait(t)
                if info.state != rt.REQ_DONE:
                    failed.append((i, info.status))
                srv.release(t)
                if i >= w:
                    lat.append(info.t_done - target)
                    done.append(info.t_done)
                    recs.append({"target": target, "t_submit": info.t_submit, "t_launch": info.t_launch,
                                 "t_done": info.t_done, "batch": info.batch_size, "side": side})
                i += 1

        th = _th.Thread(target=consume, daemon=True)
        th.start()
        t0 = time.perf_counter() + 0.05
        first = None
        for k in range(n):
            target = t0 + trace[k]["t"] / speed
            wait_until(target)
            tickets.put((target, srv.submit(reqs[k]), reqs[k].width))
            if k == w:
                first = target
        tickets.put(None)
        th.join()
        if failed:
            raise RuntimeError(f"requests failed: {failed[:5]}")
        st = srv.stats()
        srv.close()
        torch.cuda.synchronize()
        # the device counter covers every request, warm-up included: scale to the measured ones
        samples = int(counter.item()) * (n - w) / n
        out = summarize(lat, int(samples), first, max(done), n - w)
        out.update({"pool_bytes": int(st.pool_bytes), "pool_peak_bytes": int(st.pool_peak),
                    "batches": int(st.batches), "mean_batch": round(n / max(int(st.batches), 1), 2),
                    "breakdown": serve_breakdown(recs)})
        return out

    def serial(speed=1.0, n=None):
        n = n or n_req
        tfs = rt.TransferFunction(reqs[0].tf_rgba, 0.0, 4095.0)
        counter = torch.zeros(1, dtype=torch.int64, device="cuda")
        t0 = time.perf_counter() + 0.05
        lat, done, targets = [], [], []
        for k in range(n):
            r = reqs[k]
            target = t0 + trace[k]["t"] / speed
            wait_until(target)
            tfs.update(r.tf_rgba)
            if k == warm and speed == 1.0:
                counter.zero_()
            rt.render(ex.volumes[r.volume_id], tfs, r.camera, r.width, r.height, 0.5, 0.99, sample_counter=counter,
                      skip_empty=True)
            torch.cuda.synchronize()
            t = time.perf_counter()
            lat.append(t - target)
            done.append(t)
            targets.append(target)
        w = warm if speed == 1.0 else 0
        if speed != 1.0:
            pass
        return summarize(lat[w:], int(counter.item()), targets[w], done[-1], n - w)

    resident = ex.resident_bytes()
    loose = served(resident + (4 << 30))
    tight = served(resident + (64 << 20))
    nat_loose = served_native(4 << 30)
    nat_tight = served_native(64 << 20)
    ser = serial()
    fast_n = min(1000, n_req)
    sat = {"speedup_of_arrivals": 20, "served": served(resident + (4 << 30), 20.0, fast_n),
           "native": served_native(4 << 30, 20.0, fast_n), "serial": serial(20.0, fast_n)}
    line = _contract(f"p50/p99 render latency (ms), Poisson 200 req/s over 16 resident 12-bit volumes stored as "
                     f"{args.storage}, continuous batching (native server; value = p99)", nat_loose["p99_ms"], "ms", args, nat_loose["mean_ms"],
                     "f32",
                     {"workload": f"serve-poisson200-16vol-{args.storage}-{args.layout}", "volumes": len(dims),
                      "sizes": W.BATCH_SIZES, "storage": args.storage, "layout": args.layout,
                      "batch_form": args.batch_form, "tile_order": args.tile_order or 2,
                      "requests": n_req, "warmup_requests": warm, "image_sides": [256, 1024], "streams": 3,
                      "max_batch": 64, "step_vox": 0.5, "alpha_cutoff": 0.99, "tf_entries": 4096,
                      "skip_empty": True},
                     resident_bytes=resident, native_loose_pool=nat_loose, native_tight_pool=nat_tight,
                     python_server_loose_budget=loose, python_server_tight_budget=tight,
                     serial_plain=ser, saturation=sat)
    line["higher_is_better"] = False
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--probe-copy", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="orbit and batch: keep the plans' default launch "
                    "shape (8x8 tiles, 12 waves; 16 with skipping)")
    ap.add_argument("--only", choices=["batch", "plain", "graph", "skip"], default=None,
                    help="time one launch form only (for profiling); skip = the graph form with empty-space "
                         "skipping")
    ap.add_argument("--shape-skip", default=None, help="orbit: launch shape TWxTHxWAVES of the skipping form "
                    "(default: --shape, or its own autotuned shape); up to 16 waves, against 12 for fixed steps")
    ap.add_argument("--shape", default=None, help="orbit: fixed launch shape TWxTHxWAVES (e.g. 4x16x16) "
                                                  "instead of the autotuner's")
    ap.add_argument("--ingest-traffic", default=None, metavar="DIR",
                    help="read rocprofv3 FETCH_SIZE/WRITE_SIZE CSVs from DIR/{fetch,write,copy_fetch,copy_write} "
                         "and record the orbit kernel's HBM bytes per launch in profiles/traffic.json")
    ap.add_argument("--traffic-key", default="brain-orbit-36x512x512-u12-quads:graph",
                    help="workload:form the ingested counters belong to")
    ap.add_argument("--valu-kernel", default="march_batch_kernel<6, 4>",
                    help="kernel whose counters --ingest-valu reads (name and template arguments as the "
                         "profiler prints them)")
    ap.add_argument("--ingest-valu", default=None, metavar="DIR",
                    help="read a rocprofv3 SQ/GRBM counter CSV from DIR/valu and record the orbit kernel's VALU "
                         "issue figures in profiles/valu_counters.json (key --traffic-key; needs --valu-samples)")
    ap.add_argument("--valu-samples", type=int, default=0, help="composited samples per launch (for --ingest-valu)")
    ap.add_argument("--requests", type=int, default=4000, help="serve workload: number of requests")
    ap.add_argument("--workload", choices=["orbit", "precision", "batch", "serve", "projection"], default="orbit",
                    help="orbit: 36 views of the 256x256x160 u16 phantom at 512^2 (default); precision: "
                         "the same phantom as u16/f16/8-bit bricks at 1024^2, step 0.25; batch: 32 uneven "
                         "volumes x 4 views in one launch vs 128 launches; serve: Poisson request stream; "
                         "projection: the orbit under every ray function (projections, thresholding, "
                         "iso-surface)")
    ap.add_argument("--batch-form", type=int, choices=[0, 1, 2], default=0,
                    help="serve: the servers' batch plans take the latency form by batch size (0), never (1) or "
                         "always (2)")
    ap.add_argument("--tile-order", type=int, choices=[0, 1, 2], default=0,
                    help="serve: tile order of the executor's plans (0 = its default, spread; 1 compact; 2 spread)")
    ap.add_argument("--layout", choices=["cells", "poly", "linear", "quads"], default=None,
                    help="device layout of the orbit volume (and of every volume of the batch workload); "
                         "default: quad bricks for u12/u16 storage, cells for u15")
    ap.add_argument("--storage", choices=["u16", "u15", "u12"], default="u12",
                    help="device storage of the 12-bit uint16 phantoms, all exact for them (u15: x-pairs as "
                         "differences, images bit-identical to u16; u12: halves of value-2048, images equal to "
                         "u16 within binary32 rounding); the orbit compares its images with u16 storage in the "
                         "run; the precision workload always measures its own list")
    args = ap.parse_args()
    if args.layout is None:
        args.layout = "cells" if args.storage == "u15" else "quads"

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py renders on exactly one GPU: the raycaster has no multi-GPU path "
              "(views would shard across GPUs with no exchange); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1211_5595_amd as rt
    import workloads as W

    if args.probe_copy:
        probe_copy()
        return
    if args.ingest_traffic:
        return ingest_traffic(args.ingest_traffic, args.traffic_key)
    if args.ingest_valu:
        if args.valu_samples <= 0:
            raise SystemExit("--ingest-valu needs --valu-samples")
        return ingest_valu(args.ingest_valu, args.traffic_key, args.valu_samples, kernel=args.valu_kernel)
    if args.workload == "precision":
        return bench_precision(args)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "projection":
        return bench_projection(args)

    cfg = W.CONFIG_BRAIN
    vs, ts = cfg["volume"], cfg["tf"]
    width, height, step, cutoff, n_views = cfg["width"], cfg["height"], cfg["step_vox"], cfg["cutoff"], cfg["n_views"]
    vol_np = W.phantom_brain(vs.seed, dims=vs.dims, spacing=vs.spacing)
    tf_np = W.random_tf(ts.K, ts.seed, alpha_max=ts.alpha_max)
    cams = W.orbit_cameras(vs.dims, vs.spacing, n_views)

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    layout = _layout(rt, args)
    storage = _storage(rt, args)
    vol = rt.Volume(vol_np, vs.spacing, storage=storage, layout=layout)
    tf = rt.TransferFunction(tf_np, ts.vmin, ts.vmax)
    outs = [torch.empty((height, width, 4), dtype=torch.float32, device="cuda") for _ in range(n_views)]
    jobs = [rt.Job(vol, tf, cam, width, height, step, cutoff, out=o) for cam, o in zip(cams, outs)]
    tuned = None
    def parse_shape(text):
        tw, th, wv = (int(x) for x in text.split("x"))
        return dict(tile=(tw, th), waves_per_block=wv)

    shape_skip = parse_shape(args.shape_skip) if args.shape_skip else None
    if args.shape:
        shape = parse_shape(args.shape)
    elif not args.no_autotune:
        from paper_1211_5595_amd import autotune
        tuned = autotune.tune_launch(vol, tf, cams, width, height, step, cutoff, reps=3)
        shape = dict(tile=tuple(tuned["tile"]), waves_per_block=tuned["waves_per_block"])
    else:
        shape = dict(tile=(8, 8), waves_per_block=12)
    plan = rt.BatchPlan(n_views, storage, layout=layout, **shape)

    # untimed counting pass, with per-pixel counts for the samples per hitting ray
    counter = torch.zeros(1, dtype=torch.int64, device="cuda")
    pix = [torch.zeros((height, width), dtype=torch.int32, device="cuda") for _ in cams]
    rt.render_batch([rt.Job(vol, tf, cam, width, height, step, cutoff, out=o, pixel_counts=c)
                     for cam, o, c in zip(cams, outs, pix)], sample_counter=counter)
    torch.cuda.synchronize()
    samples_per_step = int(counter.item())
    hitting_rays = int(sum(int((c > 0).sum()) for c in pix))
    del pix
    vs_u16 = None
    if storage != rt.U16:  # the same views from 16-bit storage of the same grid
        vol16 = rt.Volume(vol_np, vs.spacing, storage=rt.U16, layout=layout)
        outs16 = rt.render_batch([rt.Job(vol16, tf, cam, width, height, step, cutoff) for cam in cams])
        torch.cuda.synchronize()
        diff = torch.stack([(a - b).abs().amax(-1) for a, b in zip(outs, outs16)])
        vs_u16 = {"bitwise_equal": all(torch.equal(a, b) for a, b in zip(outs, outs16)),
                  "max_abs_diff": float(diff.max()), "pixels_above_1e-5": int((diff > 1e-5).sum())}
        del diff

    def step_batch():
        rt.render_batch(jobs, **shape)

    def step_graph():
        plan.launch(jobs)

    step_plain = _plain_caller(rt, jobs)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    forms = {"batch": step_batch, "graph": step_graph, "plain": step_plain}
    if args.only == "skip":
        plan_s = rt.BatchPlan(n_views, storage, layout=layout, skip_empty=True, **(shape_skip or shape))
        jobs_s = [rt.Job(vol, tf, cam, width, height, step, cutoff, out=o, skip_empty=True)
                  for cam, o in zip(cams, outs)]
        forms = {"skip": lambda: plan_s.launch(jobs_s)}
    elif args.only:
        forms = {args.only: forms[args.only]}
    ms = {k: timed(fn, args.steps, args.warmup) for k, fn in forms.items()}
    if vs_u16 is not None and not args.only:  # the same launch form over the 16-bit cells, for reference
        plan16 = rt.BatchPlan(n_views, rt.U16, layout=layout, **shape)
        jobs16 = [rt.Job(vol16, tf, cam, width, height, step, cutoff, out=o) for cam, o in zip(cams, outs16)]
        ms16 = timed(lambda: plan16.launch(jobs16), args.steps, args.warmup)
        vs_u16["u16_graph_ms_per_step"] = round(ms16, 4)
        vs_u16["u16_gsamples_per_s"] = round(samples_per_step / (ms16 * 1e-3) / 1e9, 3)
        del plan16, jobs16
    if vs_u16 is not None:
        del vol16, outs16
    best = min(ms, key=ms.get)
    ms_step = ms[best]
    gsps = samples_per_step / (ms_step * 1e-3) / 1e9
    fps = n_views / (ms_step * 1e-3)

    # single-view latency of the plain per-frame renderer (enqueue -> done, device
    # clock), arguments marshalled before the timed calls
    def single_view_latency(opts, images):
        import ctypes as C
        L = rt.lib()
        calls = []
        for cam, o in zip(cams, images):
            calls.append((C.c_void_p(vol.handle), (C.c_int64 * 3)(*vol.dims), None, C.c_void_p(tf.handle),
                          C.byref(rt.make_camera(cam)), width, height, C.c_double(step), C.c_double(cutoff), None,
                          C.c_void_p(o.data_ptr()), C.byref(opts), rt._stream_ptr()))
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(3 * n_views)]
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(evs):
            a.record(stream)
            L.rt_render(*calls[k % n_views])
            b.record(stream)
        torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in evs]

    lat = []
    if not args.only:
        lat = single_view_latency(rt.make_opts(), outs)  # rt_render's own default launch shape

    # roofline of the dominant kernel.  The binding resource is vector-ALU
    # instruction issue: the VALU lane-slots the launch issues per second
    # against the non-packed issue peak.  The issued count is SQ_INSTS_VALU x
    # 64 per launch, counted by rocprofv3 on the same kernel sources (a fixed
    # property of kernel and workload: the same samples take the same
    # branches), divided by the composited samples to give the figure per
    # sample.  Without such counters the compositing loop of the built code
    # object stands in, every sample taking the colour block (an upper bound
    # of the loop's part that leaves out per-ray set-up).  Beside it, the
    # logical gather bytes (8 trilinear corners x 2 B per sample + 16 B per
    # output pixel; the caches serve most of them, so they are not a
    # ceiling) and the fabric bytes the counters measured.
    algo_bytes = samples_per_step * 16 + n_views * width * height * 16
    launches_per_step = 1 if best in ("batch", "graph", "skip") else n_views
    bytes_per_launch = algo_bytes / launches_per_step
    samples_per_launch = samples_per_step / launches_per_step
    ms_per_launch = ms_step / launches_per_step
    workload = f"brain-orbit-36x512x512-{args.storage}-{args.layout}"
    key = workload + ":" + best
    traffic = load_traffic(key)
    roof = None
    if best != "skip":  # skipped samples are never gathered: no per-sample roofline for that form
        from paper_1211_5595_amd import isa
        batch_form = best in ("batch", "graph")
        kname = "march_batch_kernel" if batch_form else "march_plain_kernel"
        try:  # the loop's counts come from the ROCm LLVM tools; the line does not depend on them
            lp = isa.loop_profile(rt.LIB_PATH, storage, layout, kname)
        except (OSError, subprocess.SubprocessError, ValueError) as exc:
            print(f"loop profile unavailable: {exc}", file=sys.stderr)
            lp = None
        cnt = load_valu(key)
        if cnt is not None:
            vps = cnt["sq_insts_valu"] * 64.0 / samples_per_launch
            vps_from = ("VALU lane-slots issued per composited sample: rocprofv3 SQ_INSTS_VALU x 64 per launch "
                        "(profiles/valu_counters.json, same kernel sources) / samples per launch")
        elif lp is not None:
            vps = lp["valu_per_sample"]
            vps_from = ("VALU instructions per compositing sample of the loop in the built gfx950 code object "
                        "(paper_1211_5595_amd/isa.py); no counters for these kernel sources")
        else:
            raise SystemExit(f"no VALU counters and no compositing loop found for {kname}<{storage}, {layout}>")
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        roof = valu_roofline(samples_per_launch, ms_per_launch, vps, cus)
        gb = lambda b: round(b / (ms_per_launch * 1e-3) / 1e9, 1)
        roof.update({
            "traffic": traffic,
            "kernel": kname + "<" + args.storage + ">",
            "valu_per_sample": round(vps, 3),
            "valu_per_sample_from": vps_from,
            "loop": None if lp is None else {
                "valu_per_compositing_sample": lp["valu_per_sample"],
                "valu_per_transparent_sample": lp["valu_per_transparent_sample"],
                "note": "the compositing loop of the built code object; a wave whose opacities are all zero "
                        "skips the colour block"},
            "samples_per_launch": int(samples_per_launch),
            "limiter": _limiter(best, args.storage, args.layout),
            "logical_gather": {"bytes_per_launch": int(bytes_per_launch), "GB_per_s": gb(bytes_per_launch),
                               "frac_of_hbm_peak": round(bytes_per_launch / (ms_per_launch * 1e-3) / 1e9
                                                         / PEAK_HBM_GBS, 4),
                               "note": "8 corners x 2 B per sample + 16 B per pixel; L1/L2 serve most of "
                                       "these gathers, so this figure is not a ceiling and can exceed 1"},
            "fabric": None if traffic is None else {
                "bytes_per_launch": traffic, "GB_per_s": gb(traffic),
                "frac_of_hbm_peak": round(traffic / (ms_per_launch * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                "note": "FETCH_SIZE x 2 + WRITE_SIZE x 1 per launch (scales from a plain copy); reads served "
                        "by the Infinity Cache count as fetched"},
        })
        if cnt is not None:
            roof["counters"] = {k: cnt.get(k) for k in ("sq_insts_valu", "valu_wave_insts_per_sample",
                                                       "lane_utilisation", "issue_frac_of_busy_cycles",
                                                       "issue_frac_at_peak_clock", "clock_GHz")}

    line = {
        "metric": "ray samples/sec (G/s) + fps at 512x512 over 256x256x160; p50/p99 render latency",
        "value": round(gsps, 3),
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "volume": list(vs.dims), "spacing": list(vs.spacing),
                   "source_dtype": "u16 (12-bit range)", "storage": args.storage,
                   "image": [width, height], "views": n_views, "step_vox": step, "alpha_cutoff": cutoff,
                   "tf_entries": ts.K, "launch": best, "layout": args.layout, "tile": list(shape["tile"]),
                   "waves_per_block": shape["waves_per_block"]},
        "autotune": tuned,
        "images_vs_u16_storage": vs_u16,
        "fps": round(fps, 1),
        "samples_per_step": samples_per_step,
        "hitting_rays_per_step": hitting_rays,
        "mean_samples_per_hitting_ray": round(samples_per_step / max(hitting_rays, 1), 1),
        "ms_per_step_by_form": {k: round(v, 4) for k, v in ms.items()},
        "gsamples_per_s_by_form": {k: round(samples_per_step / (v * 1e-3) / 1e9, 3) for k, v in ms.items()},
        "latency_ms": {"single_view_p50": percentile(lat, 50), "single_view_p99": percentile(lat, 99),
                       "orbit_step": round(ms_step, 4)} if lat else None,
        "roofline": roof,
    }
    if roof is not None and not args.only:  # what a plain device copy achieves on this GPU
        roof["achievable_copy_GBps"] = round(probe_copy(1.0, 10, quiet=True), 1)
    # exact empty-space skipping over the same views: same images, same
    # composited-sample count, fewer samples gathered; reported beside the
    # fixed-step figure, never as it
    if not args.only:
        shape_s = shape_skip or shape
        if tuned is not None and shape_skip is None:
            from paper_1211_5595_amd import autotune
            t_s = autotune.tune_launch(vol, tf, cams, width, height, step, cutoff, reps=3, skip_empty=True)
            shape_s = dict(tile=tuple(t_s["tile"]), waves_per_block=t_s["waves_per_block"])
        plan_s = rt.BatchPlan(n_views, storage, layout=layout, skip_empty=True, **shape_s)
        outs_s = [torch.empty_like(o) for o in outs]
        jobs_s = [rt.Job(vol, tf, cam, width, height, step, cutoff, out=o, skip_empty=True)
                  for cam, o in zip(cams, outs_s)]
        ms_s = timed(lambda: plan_s.launch(jobs_s), args.steps, args.warmup)
        plan.launch(jobs)
        torch.cuda.synchronize()
        same = all(torch.equal(a, b) for a, b in zip(outs, outs_s))
        lat_s = single_view_latency(rt.make_opts(skip_empty=True, **shape_s), outs_s)
        line["skip_empty"] = {"ms_per_step": round(ms_s, 4), "fps": round(n_views / (ms_s * 1e-3), 1),
                              "speedup_vs_fixed_step": round(ms_step / ms_s, 3),
                              "composited_gsamples_per_s": round(samples_per_step / (ms_s * 1e-3) / 1e9, 3),
                              "images_bitwise_equal": bool(same), "tile": list(shape_s["tile"]),
                              "waves_per_block": shape_s["waves_per_block"],
                              "single_view_p50_ms": percentile(lat_s, 50), "single_view_p99_ms": percentile(lat_s, 99)}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(vol_np, tf_np, cams, vs.spacing, width, height, step, cutoff, ts.vmax,
                                            args.cpu_budget)
        line["small_config"] = small_config()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
