"""Autotuner for the marcher's launch shape and a volume's storage and layout.

Tunables: the ray tile of one wavefront (8x8, 16x4, 4x16, 32x2 pixels), the
wavefronts per workgroup (4, 8, 12 for fixed steps; 4, 8, 16 with skipping) and, per volume at creation, the storage
layout (cell-packed, quad bricks for 16- and 12-bit data, polynomial cells for integer data, or linear; for 8-bit
brick storage the brick edge 8, 16 or 32) or, for integer data, the storage
type among the encodings that hold the grid exactly (tune_storage).  Tile shape and wavefronts never
change a pixel; the cell-packed, quad-brick and linear layouts render the same
image bit for bit, and the polynomial layout evaluates the same interpolant in another
rounding order (within the same tolerance of the exact result), so the choice
is speed.  Each candidate is timed on
representative views with device events; results are cached in a JSON file
keyed by GPU architecture, storage type, layout, volume size class and image
size class.
"""
from __future__ import annotations

import json
import math
import os
import threading
from typing import Callable, Dict, Iterable, List, Optional, Sequence, Tuple

TILES: List[Tuple[int, int]] = [(8, 8), (16, 4), (4, 16), (32, 2)]
# wavefronts per workgroup: the fixed-step batched kernel takes at most 12,
# the skipping one 16
WAVES: List[int] = [4, 8, 12]
WAVES_SKIP: List[int] = [4, 8, 16]
DEFAULT_CACHE = os.environ.get("RT_AUTOTUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "rtvol", "autotune.json"))


def size_class(n: int) -> int:
    """log2 bucket of a count (voxels or pixels)."""
    return int(math.floor(math.log2(max(int(n), 1))))


def launch_key(arch: str, storage: int, layout: int, dims: Sequence[int], width: int, height: int,
               skip_empty: bool = False) -> str:
    key = f"{arch}|s{storage}|l{layout}|v{size_class(dims[0] * dims[1] * dims[2])}|i{size_class(width * height)}"
    return key + ("|skip" if skip_empty else "")


class Cache:
    """A small JSON cache, written atomically."""

    def __init__(self, path: str = DEFAULT_CACHE):
        self.path = path
        self._lock = threading.Lock()
        self.data: Dict[str, dict] = {}
        try:
            with open(path) as f:
                self.data = json.load(f)
        except (OSError, ValueError):
            self.data = {}

    def get(self, key: str) -> Optional[dict]:
        return self.data.get(key)

    def put(self, key: str, value: dict):
        with self._lock:
            self.data[key] = value
            d = os.path.dirname(self.path)
            if d:
                os.makedirs(d, exist_ok=True)
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.data, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def pick_best(candidates: Iterable, measure: Callable[[object], float]) -> Tuple[object, Dict[str, float]]:
    """Measure every candidate (milliseconds, lower is better) and return the
    fastest with the table of timings."""
    table, best, best_ms = {}, None, float("inf")
    for c in candidates:
        ms = float(measure(c))
        table[str(c)] = ms
        if ms < best_ms:
            best, best_ms = c, ms
    return best, table


def _gpu_arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def _time_ms(fn, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def launch_candidates(skip_empty: bool = False, tiles: Sequence[Tuple[int, int]] = TILES,
                      waves: Optional[Sequence[int]] = None) -> List[Tuple[Tuple[int, int], int]]:
    """(tile, wavefronts per workgroup) pairs the launch tuner times."""
    if waves is None:
        waves = WAVES_SKIP if skip_empty else WAVES
    return [(tuple(t), int(w)) for t in tiles for w in waves]


def tune_launch(volume, tf, cameras, width: int, height: int, step_vox: float = 0.5, alpha_cutoff: float = 0.99,
                reps: int = 3, tiles: Sequence[Tuple[int, int]] = TILES, waves: Optional[Sequence[int]] = None,
                cache: Optional[Cache] = None, force: bool = False, skip_empty: bool = False) -> dict:
    """Choose tile shape and wavefronts per workgroup for batched renders of
    `cameras` (representative views) of this volume at width x height (with
    empty-space skipping when skip_empty: that kernel has its own best shape).
    Each candidate is timed as it would run: a batch plan (the persistent
    launch captured in a graph) per shape, replayed."""
    from . import BatchPlan, Job
    import torch
    key = launch_key(_gpu_arch(), volume.storage, volume.layout, volume.dims, width, height, skip_empty)
    if cache is not None and not force:
        hit = cache.get(key)
        if hit is not None:
            return hit
    outs = [torch.empty((height, width, 4), dtype=torch.float32, device=volume.buf.device) for _ in cameras]
    jobs = [Job(volume, tf, c, width, height, step_vox, alpha_cutoff, out=o, skip_empty=skip_empty)
            for c, o in zip(cameras, outs)]

    def measure(c):
        plan = BatchPlan(len(jobs), volume.storage, tile=c[0], waves_per_block=c[1], layout=volume.layout,
                         skip_empty=skip_empty)
        try:
            return _time_ms(lambda: plan.launch(jobs), reps)
        finally:
            torch.cuda.synchronize()
            plan.close()

    best, table = pick_best(launch_candidates(skip_empty, tiles, waves), measure)
    result = {"tile": list(best[0]), "waves_per_block": best[1], "ms": table[str(best)], "timings_ms": table,
              "key": key, "timed": "batch plan (graph replay)"}
    if cache is not None:
        cache.put(key, result)
    return result


def tune_batch(jobs, storage: int, layout: int, reps: int = 2, tiles: Sequence[Tuple[int, int]] = TILES,
               waves: Optional[Sequence[int]] = None, cache: Optional[Cache] = None, force: bool = False,
               skip_empty: bool = False) -> dict:
    """Choose tile shape and wavefronts per workgroup for one batch of jobs
    (views of several volumes and sizes) as it runs: a persistent batch plan
    per candidate shape, replayed on the whole batch.  The cache key is the
    storage type, layout, job count and total pixels (in powers of two)."""
    from . import BatchPlan
    import torch
    pixels = sum(j.width * j.height for j in jobs)
    key = (f"{_gpu_arch()}|batch|s{storage}|l{layout}|n{size_class(len(jobs))}|p{size_class(pixels)}"
           + ("|skip" if skip_empty else ""))
    if cache is not None and not force:
        hit = cache.get(key)
        if hit is not None:
            return hit

    def measure(c):
        plan = BatchPlan(len(jobs), storage, tile=c[0], waves_per_block=c[1], layout=layout, skip_empty=skip_empty,
                         batch_form=1)
        try:
            return _time_ms(lambda: plan.launch(jobs), reps)
        finally:
            torch.cuda.synchronize()
            plan.close()

    best, table = pick_best(launch_candidates(skip_empty, tiles, waves), measure)
    result = {"tile": list(best[0]), "waves_per_block": best[1], "ms": table[str(best)], "timings_ms": table,
              "key": key, "timed": "batch plan (graph replay) of the whole batch"}
    if cache is not None:
        cache.put(key, result)
    return result


def exact_storages(values) -> List[Tuple[int, int]]:
    """(storage, layout) pairs that hold an integer grid without loss: 8-bit
    data as u8 (any integer layout) or u16; 16-bit data as u16, and also as
    15-bit difference cells when its maximum is at most 32767 (cell layout)
    and as 12-bit halves when it is at most 4096 (cells or quad bricks).  Float data
    has no alternative to its own type here (empty list)."""
    import numpy as np
    from . import LAYOUT_CELLS, LAYOUT_LINEAR, LAYOUT_POLY, LAYOUT_QUADS, U8, U12, U15, U16
    dt = np.asarray(values).dtype
    if dt not in (np.uint8, np.uint16):
        return []
    vmax = int(np.asarray(values).max()) if np.asarray(values).size else 0
    out = [(U16, LAYOUT_CELLS), (U16, LAYOUT_POLY), (U16, LAYOUT_LINEAR), (U16, LAYOUT_QUADS)]
    if dt == np.uint8:
        out = [(U8, LAYOUT_CELLS), (U8, LAYOUT_POLY), (U8, LAYOUT_LINEAR)] + out
    if vmax <= 32767:
        out.append((U15, LAYOUT_CELLS))
    if vmax <= 4096:
        out += [(U12, LAYOUT_CELLS), (U12, LAYOUT_QUADS)]
    return out


def tune_storage(values, spacing, tf, cameras, width: int, height: int, step_vox: float = 0.5,
                 alpha_cutoff: float = 0.99, reps: int = 3, cache: Optional[Cache] = None,
                 force: bool = False) -> dict:
    """Choose the device storage type and layout of an integer volume among the
    exact encodings (exact_storages) by timing batched renders of
    representative views.  Every candidate holds the same grid; u15 cells
    render bit for bit as u16 cells, the polynomial layout and u12 cells
    evaluate the same interpolant in another rounding order (within the same
    tolerance of the exact result)."""
    from . import Job, Volume, render_batch
    import torch
    import numpy as np
    nz, ny, nx = values.shape
    cands = exact_storages(values)
    if not cands:
        raise ValueError("tune_storage needs uint8 or uint16 data")
    key = (f"{_gpu_arch()}|storage|d{np.asarray(values).dtype}|m{int(np.asarray(values).max()).bit_length()}"
           f"|v{size_class(nx * ny * nz)}|i{size_class(width * height)}")
    if cache is not None and not force:
        hit = cache.get(key)
        if hit is not None:
            return hit

    def measure(c):
        vol = Volume(values, spacing, storage=c[0], layout=c[1])
        outs = [torch.empty((height, width, 4), dtype=torch.float32, device=vol.buf.device) for _ in cameras]
        jobs = [Job(vol, tf, cam, width, height, step_vox, alpha_cutoff, out=o) for cam, o in zip(cameras, outs)]
        ms = _time_ms(lambda: render_batch(jobs), reps)
        measure.bytes[str(c)] = vol.nbytes
        return ms
    measure.bytes = {}
    best, table = pick_best(cands, measure)
    result = {"storage": best[0], "layout": best[1], "ms": table[str(best)], "timings_ms": table,
              "bytes": measure.bytes, "key": key}
    if cache is not None:
        cache.put(key, result)
    return result


def tune_layout(values, spacing, storage: int, tf, cameras, width: int, height: int, step_vox: float = 0.5,
                alpha_cutoff: float = 0.99, reps: int = 3, candidates: Optional[Sequence[Tuple[int, int]]] = None,
                cache: Optional[Cache] = None, force: bool = False) -> dict:
    """Choose the storage layout (and brick edge for 8-bit brick storage) of a
    volume by timing batched renders of representative views.  Candidates are
    (layout, brick) pairs."""
    from . import (Job, LAYOUT_BRICKS, LAYOUT_CELLS, LAYOUT_LINEAR, LAYOUT_POLY, LAYOUT_QUADS, U8, U12, U16,
                   U8_BRICKSCALED, Volume, render_batch)
    import torch
    nz, ny, nx = values.shape
    key = f"{_gpu_arch()}|layout|s{storage}|v{size_class(nx * ny * nz)}|i{size_class(width * height)}"
    if cache is not None and not force:
        hit = cache.get(key)
        if hit is not None:
            return hit
    if candidates is None:
        if storage == U8_BRICKSCALED:
            candidates = [(l, b) for l in (LAYOUT_CELLS, LAYOUT_BRICKS) for b in (8, 16, 32)]
        elif storage == U16:
            candidates = [(LAYOUT_CELLS, 0), (LAYOUT_POLY, 0), (LAYOUT_LINEAR, 0), (LAYOUT_QUADS, 0)]
        elif storage == U8:
            candidates = [(LAYOUT_CELLS, 0), (LAYOUT_POLY, 0), (LAYOUT_LINEAR, 0)]
        elif storage == U12:
            candidates = [(LAYOUT_CELLS, 0), (LAYOUT_QUADS, 0)]
        else:
            candidates = [(LAYOUT_CELLS, 0), (LAYOUT_LINEAR, 0)]

    def measure(c):
        vol = Volume(values, spacing, storage=storage, layout=c[0], brick=c[1])
        outs = [torch.empty((height, width, 4), dtype=torch.float32, device=vol.buf.device) for _ in cameras]
        jobs = [Job(vol, tf, cam, width, height, step_vox, alpha_cutoff, out=o) for cam, o in zip(cameras, outs)]
        ms = _time_ms(lambda: render_batch(jobs), reps)
        measure.bytes[str(c)] = vol.nbytes
        return ms
    measure.bytes = {}
    best, table = pick_best(candidates, measure)
    result = {"layout": best[0], "brick": best[1], "ms": table[str(best)], "timings_ms": table,
              "bytes": measure.bytes, "key": key}
    if cache is not None:
        cache.put(key, result)
    return result
