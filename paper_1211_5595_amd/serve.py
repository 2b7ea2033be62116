"""Render server: resident volumes, admission by HBM budget, continuous batching.

The paper asks for rendering "at interactive speed" that is "robust to mass
data" (Sections 1 and 4.3).  This module serves render requests against
volumes kept resident in device memory:

* requests are admitted first-in first-out while the bytes they need (output
  image and transfer-function table) plus the resident volumes stay within an
  HBM budget; a request that could never fit is rejected at once;
* every scheduler tick gathers the admitted requests into one batch and
  launches it as a single persistent batched render on a free stream from a
  small pool, so requests that arrive while others run are admitted as soon as
  a stream and memory free up, and several batches run on the device at once;
* a future per request resolves with the image when its batch's completion
  event fires; latency runs from submission to that moment.

The scheduling logic is independent of the device: it talks to an executor
(``GpuExecutor`` renders through the C ABI; tests drive the same scheduler
with a scripted executor and a fake clock).
"""
from __future__ import annotations

import collections
import ctypes
import dataclasses
import threading
import time
from typing import Any, Callable, Deque, Dict, List, Optional, Sequence

import numpy as np

__all__ = ["RenderRequest", "RenderFuture", "Server", "GpuExecutor", "RejectedError", "RequestTimeout"]


class RejectedError(RuntimeError):
    """The request can never fit the HBM budget (or names an unknown volume)."""


class RequestTimeout(TimeoutError):
    """The request waited in the queue past its deadline."""


@dataclasses.dataclass
class RenderRequest:
    volume_id: Any
    camera: Any
    width: int
    height: int
    tf_rgba: np.ndarray          # K x 4 float32 in [0, 1]
    vmin: float = 0.0
    vmax: float = 4095.0
    step_vox: float = 0.5
    alpha_cutoff: float = 0.99
    bg: Sequence[float] = (0.0, 0.0, 0.0, 0.0)
    deadline: Optional[float] = None   # absolute time on the server clock; None = wait forever
    ray_function: int = 0              # rt_ray_function (compositing by default)
    iso_value: float = 0.0             # iso-value, or the low end of a threshold window
    iso_high: float = 0.0              # high end of a threshold window
    opacity_unit_distance: float = 0.0 # > 0: opacity correction to this distance (mm)


class RenderFuture:
    def __init__(self, req: RenderRequest, t_submit: float):
        self.request = req
        self.t_submit = t_submit
        self.t_done: Optional[float] = None
        self._event = threading.Event()
        self._result = None
        self._error: Optional[BaseException] = None
        self._cancelled = False
        self.samples: Optional[int] = None

    def cancel(self) -> bool:
        """Cancel a request that has not been launched yet."""
        if self._event.is_set():
            return False
        self._cancelled = True
        return True

    @property
    def cancelled(self) -> bool:
        return self._cancelled

    def done(self) -> bool:
        return self._event.is_set()

    def result(self, timeout: Optional[float] = None):
        if not self._event.wait(timeout):
            raise TimeoutError("render not finished")
        if self._error is not None:
            raise self._error
        return self._result

    @property
    def latency(self) -> Optional[float]:
        return None if self.t_done is None else self.t_done - self.t_submit

    def _finish(self, result, t_done: float, error: Optional[BaseException] = None):
        self._result, self._error, self.t_done = result, error, t_done
        self._event.set()


class Server:
    """Scheduler over an executor.  ``budget_bytes`` bounds resident volumes
    plus the bytes of admitted, unfinished requests."""

    def __init__(self, executor, budget_bytes: int, max_batch: int = 64,
                 clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self.clock = clock
        self._lock = threading.Lock()
        self._queue: Deque[RenderFuture] = collections.deque()
        self._inflight: List[tuple] = []        # (token, futures, bytes)
        self.inflight_bytes = 0
        self.peak_bytes = 0
        self.completed: List[RenderFuture] = []
        self.batches = 0
        self._thread: Optional[threading.Thread] = None
        self._stop = threading.Event()
        self._wake = threading.Condition(self._lock)  # signalled by submit() and stop()

    # ---- requests -------------------------------------------------------
    def submit(self, req: RenderRequest) -> RenderFuture:
        fut = RenderFuture(req, self.clock())
        if not self.ex.has_volume(req.volume_id):
            fut._finish(None, self.clock(), RejectedError(f"unknown volume {req.volume_id!r}"))
            return fut
        need = self.ex.request_bytes(req)
        if self.ex.resident_bytes() + need > self.budget:
            fut._finish(None, self.clock(), RejectedError(
                f"request needs {need} B; budget {self.budget} B leaves "
                f"{self.budget - self.ex.resident_bytes()} B beside the resident volumes"))
            return fut
        with self._lock:
            self._queue.append(fut)
            self._wake.notify()
        return fut

    def pending(self) -> int:
        with self._lock:
            return len(self._queue) + sum(len(f) for _, f, _ in self._inflight)

    # ---- one scheduler tick --------------------------------------------
    def run_once(self) -> bool:
        """Retire finished batches, then admit and launch one batch if a slot
        is free.  Returns True if anything happened."""
        progressed = self._retire()
        now = self.clock()
        with self._lock:
            # drop cancelled and expired requests at the head of the queue and anywhere behind it
            keep: Deque[RenderFuture] = collections.deque()
            for f in self._queue:
                if f.cancelled:
                    f._finish(None, now, RuntimeError("cancelled"))
                    progressed = True
                elif f.request.deadline is not None and now > f.request.deadline:
                    f._finish(None, now, RequestTimeout("deadline passed while queued"))
                    progressed = True
                else:
                    keep.append(f)
            self._queue = keep
            if not self._queue or not self.ex.slot_free():
                return progressed
            batch, nbytes = [], 0
            resident = self.ex.resident_bytes()
            while self._queue and len(batch) < self.max_batch:
                f = self._queue[0]
                need = self.ex.request_bytes(f.request)
                if resident + self.inflight_bytes + nbytes + need > self.budget:
                    break                      # FIFO: the head waits for memory to free up
                batch.append(self._queue.popleft())
                nbytes += need
            if not batch:
                return progressed
            self.inflight_bytes += nbytes
            self.peak_bytes = max(self.peak_bytes, resident + self.inflight_bytes)
        try:
            token = self.ex.launch([f.request for f in batch])
        except Exception as e:  # device or argument error: fail the batch, keep serving
            with self._lock:
                self.inflight_bytes -= nbytes
            t = self.clock()
            for f in batch:
                f._finish(None, t, e)
            return True
        with self._lock:
            self._inflight.append((token, batch, nbytes))
        self.batches += 1
        return True

    def _retire(self) -> bool:
        done = []
        with self._lock:
            for item in list(self._inflight):
                if self.ex.poll(item[0]):
                    self._inflight.remove(item)
                    done.append(item)
        for token, futs, nbytes in done:
            t = self.clock()
            try:
                images, samples = self.ex.finish(token)
                for f, img, n in zip(futs, images, samples):
                    f.samples = n
                    f._finish(img, t)
            except Exception as e:
                for f in futs:
                    f._finish(None, t, e)
            with self._lock:
                self.inflight_bytes -= nbytes
                self.completed.extend(futs)
        return bool(done)

    # ---- background loop ------------------------------------------------
    def _idle(self, max_wait: float):
        """Nothing to do this tick.  With batches on the GPU, only yield (their
        completion is polled, and a timed sleep would add its granularity,
        tens of microseconds, to every request); otherwise block until a
        submission or stop() wakes the loop (or max_wait passes)."""
        with self._lock:
            if self._inflight:
                busy = True
            else:
                busy = False
                if not self._queue and not self._stop.is_set():
                    self._wake.wait(max_wait)
        if busy:
            time.sleep(0)

    def start(self, idle_wait: float = 1e-3):
        def loop():
            while not self._stop.is_set():
                if not self.run_once():
                    self._idle(idle_wait)
            while self.pending():
                if not self.run_once():
                    self._idle(idle_wait)
        self._stop.clear()
        self._thread = threading.Thread(target=loop, daemon=True)
        self._thread.start()

    def stop(self, drain: bool = True):
        if self._thread is None:
            return
        if not drain:
            with self._lock:
                for f in self._queue:
                    f._finish(None, self.clock(), RuntimeError("server stopped"))
                self._queue.clear()
        with self._lock:
            self._stop.set()
            self._wake.notify()
        self._thread.join()
        self._thread = None

    def drain(self):
        while self.pending():
            if not self.run_once():
                time.sleep(20e-6)

    def latency_stats(self, skip: int = 0) -> Dict[str, float]:
        lat = [f.latency for f in self.completed[skip:] if f.latency is not None and f._error is None]
        if not lat:
            return {}
        a = np.array(lat)
        return {"n": int(a.size), "p50_ms": float(np.percentile(a, 50) * 1e3),
                "p99_ms": float(np.percentile(a, 99) * 1e3), "mean_ms": float(a.mean() * 1e3),
                "max_ms": float(a.max() * 1e3)}


class GpuExecutor:
    """Runs batches through the C ABI: resident volumes, one batch plan
    (captured persistent launch) and one table pool per stream.  Compositing
    requests use exact empty-space skipping unless skip_empty is False (the
    images are the same either way).  tile_order is the plans' tile order
    (2, spread, by default: batches here are small and latency-bound)."""

    def __init__(self, n_streams: int = 3, max_batch: int = 64, storage: Optional[int] = None, device="cuda",
                 skip_empty: bool = True, tile_order: int = 2, layout: Optional[int] = None, batch_form: int = 0):
        import torch

        from . import BatchPlan, Job, TransferFunction, U16, LAYOUT_CELLS
        self.torch = torch
        self._Job, self._TF = Job, TransferFunction
        self.device = device
        self.storage = U16 if storage is None else storage
        self.layout = LAYOUT_CELLS if layout is None else layout
        self.volumes: Dict[Any, Any] = {}
        self._resident = 0
        self.streams = [torch.cuda.Stream(device=device) for _ in range(n_streams)]
        self.skip_empty = bool(skip_empty)
        self.plans = [BatchPlan(max_batch, self.storage, layout=self.layout, device=device, skip_empty=self.skip_empty,
                                tile_order=tile_order, batch_form=batch_form) for _ in range(n_streams)]
        # cumulative sample counters, copied to pinned host memory behind each
        # batch, so retiring a batch reads its count without a device round trip
        self.counters = [torch.zeros(1, dtype=torch.int64, device=device) for _ in range(n_streams)]
        self.host_counts = torch.zeros(n_streams, dtype=torch.int64, pin_memory=True)
        self._last_count = [0] * n_streams
        self.tf_pools: List[Dict[int, List[Any]]] = [collections.defaultdict(list) for _ in range(n_streams)]
        self.busy = [None] * n_streams
        self.max_batch = max_batch

    # volumes
    def add_volume(self, vid, values, spacing):
        from . import Volume
        v = Volume(values, spacing, storage=self.storage, layout=self.layout, device=self.device)
        self.volumes[vid] = v
        self._resident += v.nbytes
        return v

    def has_volume(self, vid) -> bool:
        return vid in self.volumes

    def resident_bytes(self) -> int:
        return self._resident

    @staticmethod
    def request_bytes(req: RenderRequest) -> int:
        from . import rt_tf_bytes
        return req.width * req.height * 16 + rt_tf_bytes(int(req.tf_rgba.shape[0]))

    # batches
    def slot_free(self) -> bool:
        return any(b is None for b in self.busy)

    def launch(self, reqs: Sequence[RenderRequest]):
        torch = self.torch
        k = self.busy.index(None)
        s = self.streams[k]
        pool = self.tf_pools[k]
        used: Dict[int, int] = collections.defaultdict(int)
        jobs = []
        with torch.cuda.stream(s):
            for r in reqs:
                K = int(r.tf_rgba.shape[0])
                lst = pool[K]
                i = used[K]
                used[K] += 1
                if i < len(lst):
                    tf = lst[i]
                    tf.update(r.tf_rgba, r.vmin, r.vmax, stream=s)
                else:
                    tf = self._TF(r.tf_rgba, r.vmin, r.vmax, stream=s, device=self.device)
                    lst.append(tf)
                out = torch.empty((r.height, r.width, 4), dtype=torch.float32, device=self.device)
                jobs.append(self._Job(self.volumes[r.volume_id], tf, r.camera, r.width, r.height, r.step_vox,
                                      r.alpha_cutoff, r.bg, out=out, skip_empty=self.skip_empty,
                                      ray_function=r.ray_function, iso_value=r.iso_value, iso_high=r.iso_high,
                                      opacity_unit_distance=r.opacity_unit_distance))
            self.plans[k].launch(jobs, sample_counter=self.counters[k], stream=s)
            self.host_counts[k:k + 1].copy_(self.counters[k], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        self.busy[k] = (ev, jobs)
        return k

    def poll(self, token) -> bool:
        return self.busy[token][0].query()

    def finish(self, token):
        ev, jobs = self.busy[token]
        ev.synchronize()
        self.busy[token] = None
        total = int(self.host_counts[token])
        n, self._last_count[token] = total - self._last_count[token], total
        # per-request counts are not tracked; the batch total is attributed evenly for statistics
        per = [n // len(jobs)] * len(jobs)
        return [j.out for j in jobs], per


_FLOAT_P = ctypes.POINTER(ctypes.c_float)


class NativeServer:
    """The library's own serving runtime (rt_serve.h): admission against an
    image pool, continuous batching onto n_streams streams and the request
    loop all run in a native server thread; Python only marshals requests.

    image_pool_bytes is the admission budget: a request holds its image
    (W*H*16 bytes) in the pool from admission until it is released (result()
    copies the image out and releases it).  The arena (workspaces, table slots
    and the pool) is one device allocation made here and owned by this object.
    sample_counter: an optional int64 device tensor every batch adds its
    composited samples to.
    """

    def __init__(self, image_pool_bytes: int, n_streams: int = 3, max_batch: int = 64, storage: Optional[int] = None,
                 skip_empty: bool = True, tile_order: int = 2, device="cuda", layout: Optional[int] = None,
                 batch_form: int = 0, sample_counter=None):
        import torch

        from . import (LAYOUT_CELLS, U16, make_opts, rt_server_arena_bytes, rt_server_create)
        self.torch = torch
        self.device = device
        self.storage = U16 if storage is None else storage
        self.layout = LAYOUT_CELLS if layout is None else layout
        nbytes = rt_server_arena_bytes(n_streams, max_batch, image_pool_bytes)
        self.arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        self._base = (self.arena.data_ptr() + 255) // 256 * 256
        self._shift = self._base - self.arena.data_ptr()
        torch.cuda.synchronize(device)
        self.handle = rt_server_create(n_streams, max_batch, self.storage, self.layout,
                                       make_opts(skip_empty=skip_empty, tile_order=tile_order, batch_form=batch_form,
                                                 sample_counter=sample_counter),
                                       self._base, nbytes, image_pool_bytes)
        self.volumes: Dict[Any, Any] = {}
        self._resident = 0

    # volumes
    def add_volume(self, vid, values, spacing):
        from . import Volume
        v = Volume(values, spacing, storage=self.storage, layout=self.layout, device=self.device)
        self.torch.cuda.synchronize(self.device)
        self.volumes[vid] = v
        self._resident += v.nbytes
        return v

    def resident_bytes(self) -> int:
        return self._resident

    # requests
    def submit(self, req: RenderRequest) -> int:
        """Queue a request; returns its ticket.  Raises InvalidArgument for an
        invalid request or unknown volume, OutOfMemory for an image larger
        than the whole pool."""
        from . import InvalidArgument, make_camera, rt_request, rt_server_submit
        v = self.volumes.get(req.volume_id)
        if v is None:
            raise InvalidArgument(f"unknown volume {req.volume_id!r}")
        t = req.tf_rgba
        if t.dtype != np.float32 or not t.flags.c_contiguous:
            t = np.ascontiguousarray(t, dtype=np.float32)
        # one positional constructor call: cheaper than a field-by-field fill
        r = rt_request(v.handle, t.ctypes.data_as(_FLOAT_P), t.shape[0], req.vmin, req.vmax,
                       make_camera(req.camera), req.width, req.height, req.step_vox, req.alpha_cutoff,
                       (ctypes.c_float * 4)(*req.bg), req.ray_function, req.iso_value, req.iso_high,
                       req.opacity_unit_distance)
        return rt_server_submit(self.handle, r)

    def wait(self, ticket: int, timeout: float = -1.0):
        """The request's rt_request_info once it is DONE or FAILED (or when
        timeout seconds have passed; negative = no limit)."""
        from . import rt_server_wait
        return rt_server_wait(self.handle, ticket, timeout)

    def image(self, info, width: int, height: int):
        """A view of a DONE request's image in the pool (valid until release)."""
        off = info.image_dev - self._base + self._shift
        return self.arena[off: off + width * height * 16].view(self.torch.float32).view(height, width, 4)

    def result(self, ticket: int, width: int, height: int, timeout: float = -1.0):
        """Wait, copy the image out of the pool and release the request."""
        from . import REQ_DONE, RTError, rt_server_release
        info = self.wait(ticket, timeout)
        if info.state != REQ_DONE:
            if info.state == 3:
                rt_server_release(self.handle, ticket)
                raise RTError(f"request failed with status {info.status}")
            raise TimeoutError("render not finished")
        img = self.image(info, width, height).clone()
        self.torch.cuda.current_stream(self.device).synchronize()
        rt_server_release(self.handle, ticket)
        return img

    def release(self, ticket: int):
        from . import rt_server_release
        rt_server_release(self.handle, ticket)

    def stats(self):
        from . import rt_server_get_stats
        return rt_server_get_stats(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            from . import rt_server_destroy
            rt_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
