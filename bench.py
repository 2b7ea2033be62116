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
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
KERNEL_SOURCES = ["paper_1211_5595_amd/csrc/march.hip", "paper_1211_5595_amd/csrc/ff_math.h",
                  "paper_1211_5595_amd/csrc/rt_internal.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


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
    return {"value": samples / dt / 1e9, "unit": "Gsamples/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"{n_views} of the {len(cams)} orbit views, {width}x{height}, whole images",
            "fps": n_views / dt, "seconds": dt}


def probe_copy(gib: float = 1.0, reps: int = 10):
    """Plain device copy of a known size (for counter calibration and the
    achievable-bandwidth figure)."""
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
    print(json.dumps({"probe": "copy", "bytes_read": n, "bytes_written": n, "ms": ms,
                      "GB_per_s": 2 * n / ms / 1e6}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--probe-copy", action="store_true")
    ap.add_argument("--only", choices=["batch", "plain", "graph"], default=None,
                    help="time one launch form only (for profiling)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py renders on exactly one GPU: the raycaster has no multi-GPU path in this build "
              "(views would shard across GPUs with no exchange); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1211_5595_amd as rt
    import workloads as W

    if args.probe_copy:
        probe_copy()
        return

    cfg = W.CONFIG_BRAIN
    vs, ts = cfg["volume"], cfg["tf"]
    width, height, step, cutoff, n_views = cfg["width"], cfg["height"], cfg["step_vox"], cfg["cutoff"], cfg["n_views"]
    vol_np = W.phantom_brain(vs.seed, dims=vs.dims, spacing=vs.spacing)
    tf_np = W.random_tf(ts.K, ts.seed, alpha_max=ts.alpha_max)
    cams = W.orbit_cameras(vs.dims, vs.spacing, n_views)

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    vol = rt.Volume(vol_np, vs.spacing, storage=rt.U16)
    tf = rt.TransferFunction(tf_np, ts.vmin, ts.vmax)
    outs = [torch.empty((height, width, 4), dtype=torch.float32, device="cuda") for _ in range(n_views)]
    jobs = [rt.Job(vol, tf, cam, width, height, step, cutoff, out=o) for cam, o in zip(cams, outs)]
    plan = rt.BatchPlan(n_views, rt.U16, layout=rt.LAYOUT_CELLS)

    # untimed counting pass
    counter = torch.zeros(1, dtype=torch.int64, device="cuda")
    rt.render_batch(jobs, sample_counter=counter)
    torch.cuda.synchronize()
    samples_per_step = int(counter.item())

    def step_batch():
        rt.render_batch(jobs)

    def step_graph():
        plan.launch(jobs)

    def step_plain():
        for cam, o in zip(cams, outs):
            rt.render(vol, tf, cam, width, height, step, cutoff, out=o)

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
    if args.only:
        forms = {args.only: forms[args.only]}
    ms = {k: timed(fn, args.steps, args.warmup) for k, fn in forms.items()}
    best = min(ms, key=ms.get)
    ms_step = ms[best]
    gsps = samples_per_step / (ms_step * 1e-3) / 1e9
    fps = n_views / (ms_step * 1e-3)

    # single-view latency of the plain per-frame renderer (enqueue -> done, device clock)
    lat = []
    if not args.only:
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(3 * n_views)]
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(evs):
            a.record(stream)
            rt.render(vol, tf, cams[k % n_views], width, height, step, cutoff, out=outs[k % n_views])
            b.record(stream)
        torch.cuda.synchronize()
        lat = [a.elapsed_time(b) for a, b in evs]

    # roofline of the dominant kernel: algorithmic bytes = 8 trilinear corners
    # x 2 B per sample + 16 B per output pixel, per launch
    algo_bytes = samples_per_step * 16 + n_views * width * height * 16
    launches_per_step = 1 if best in ("batch", "graph") else n_views
    bytes_per_launch = algo_bytes / launches_per_step
    ms_per_launch = ms_step / launches_per_step
    achieved = bytes_per_launch / (ms_per_launch * 1e-3) / 1e9
    workload = "brain-orbit-36x512x512-u16"
    traffic = load_traffic(workload + ":" + best)

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
        "dtype": "u16",
        "data": "synthetic",
        "config": {"workload": workload, "volume": list(vs.dims), "spacing": list(vs.spacing), "storage": "u16",
                   "image": [width, height], "views": n_views, "step_vox": step, "alpha_cutoff": cutoff,
                   "tf_entries": ts.K, "launch": best},
        "fps": round(fps, 1),
        "samples_per_step": samples_per_step,
        "ms_per_step_by_form": {k: round(v, 4) for k, v in ms.items()},
        "gsamples_per_s_by_form": {k: round(samples_per_step / (v * 1e-3) / 1e9, 3) for k, v in ms.items()},
        "latency_ms": {"single_view_p50": percentile(lat, 50), "single_view_p99": percentile(lat, 99),
                       "orbit_step": round(ms_step, 4)} if lat else None,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                     "kernel": "march_batch_kernel<u16>" if best in ("batch", "graph") else "march_plain_kernel<u16>",
                     "algorithmic_bytes_per_launch": int(bytes_per_launch)},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(vol_np, tf_np, cams, vs.spacing, width, height, step, cutoff, ts.vmax,
                                            args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
