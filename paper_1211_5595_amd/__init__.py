"""rtvol: direct volume rendering by ray casting on MI355X (gfx950).

Thin ctypes binding over the C ABI in ``include/rt.h`` (library
``librtvol.so``, built in-tree by ``paper_1211_5595_amd.build``).  Every step
of the rendering runs in the HIP kernels of that library; this module only
marshals arguments.  PyTorch provides device memory and streams.

Module-level functions carry the C names (``rt_volume_bytes``,
``rt_create_volume``, ``rt_set_transfer_function``, ``rt_render``,
``rt_render_batch``, ``rt_batch_plan_*``); the classes ``Volume``,
``TransferFunction`` and ``BatchPlan`` own the torch buffers those calls use.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

__all__ = [
    "RTError", "InvalidArgument", "OutOfMemory", "DeviceError", "Unsupported",
    "U8", "U16", "F16", "F32", "U8_BRICKSCALED", "U15", "U12", "COMPOSITE", "MIP", "XRAY", "AVERAGE", "ISO", "THRESHOLD",
    "lib", "rt_volume_bytes", "rt_create_volume", "rt_destroy_volume", "rt_tf_bytes",
    "rt_set_transfer_function", "rt_destroy_tf", "rt_render", "rt_batch_workspace_bytes",
    "rt_render_batch", "rt_render_batch_noalloc", "rt_batch_plan_create", "rt_batch_plan_launch", "rt_batch_plan_destroy",
    "rt_batch_latency_pixels",
    "rt_server_arena_bytes", "rt_server_create", "rt_server_submit", "rt_server_wait", "rt_server_release",
    "rt_server_get_stats", "rt_server_destroy", "REQ_QUEUED", "REQ_RUNNING", "REQ_DONE", "REQ_FAILED",
    "Volume", "TransferFunction", "BatchPlan", "render", "render_batch", "Job",
]

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librtvol.so")

U8, U16, F16, F32, U8_BRICKSCALED, U15, U12 = 0, 1, 2, 3, 4, 5, 6
LAYOUT_CELLS, LAYOUT_LINEAR, LAYOUT_BRICKS, LAYOUT_POLY, LAYOUT_QUADS = 0, 1, 2, 3, 4
COMPOSITE, MIP, XRAY, AVERAGE, ISO, THRESHOLD = range(6)
_DTYPE_CODE = {np.dtype(np.uint8): U8, np.dtype(np.uint16): U16, np.dtype(np.float16): F16,
               np.dtype(np.float32): F32}


class RTError(RuntimeError):
    pass


class InvalidArgument(RTError, ValueError):
    pass


class OutOfMemory(RTError, MemoryError):
    pass


class DeviceError(RTError):
    pass


class Unsupported(RTError, NotImplementedError):
    pass


_ERRORS = {1: InvalidArgument, 2: OutOfMemory, 3: DeviceError, 4: Unsupported}


class rt_camera(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("center", C.c_double * 3), ("up", C.c_double * 3),
                ("perspective", C.c_int), ("fovy_deg", C.c_double), ("ortho_half_height", C.c_double)]


class rt_render_opts(C.Structure):
    _fields_ = [("sample_counter", C.c_void_p), ("pixel_counts", C.c_void_p), ("ray_function", C.c_int),
                ("iso_value", C.c_float), ("iso_high", C.c_float), ("tile_w", C.c_int), ("tile_h", C.c_int),
                ("waves_per_block", C.c_int), ("skip_empty", C.c_int), ("tile_order", C.c_int),
                ("opacity_unit_distance", C.c_double), ("batch_form", C.c_int)]


class rt_render_job(C.Structure):
    _fields_ = [("volume", C.c_void_p), ("tf", C.c_void_p), ("camera", rt_camera), ("width", C.c_int),
                ("height", C.c_int), ("step_vox", C.c_double), ("alpha_cutoff", C.c_double),
                ("bg_rgba", C.c_float * 4), ("out_dev", C.c_void_p), ("pixel_counts", C.c_void_p),
                ("ray_function", C.c_int), ("iso_value", C.c_float), ("iso_high", C.c_float),
                ("skip_empty", C.c_int), ("opacity_unit_distance", C.c_double)]


class rt_request(C.Structure):
    _fields_ = [("volume", C.c_void_p), ("tf_rgba", C.POINTER(C.c_float)), ("tf_entries", C.c_int),
                ("tf_vmin", C.c_double), ("tf_vmax", C.c_double), ("camera", rt_camera), ("width", C.c_int),
                ("height", C.c_int), ("step_vox", C.c_double), ("alpha_cutoff", C.c_double),
                ("bg_rgba", C.c_float * 4), ("ray_function", C.c_int), ("iso_value", C.c_float),
                ("iso_high", C.c_float), ("opacity_unit_distance", C.c_double)]


class rt_request_info(C.Structure):
    _fields_ = [("state", C.c_int), ("status", C.c_int), ("image_dev", C.c_void_p), ("t_submit", C.c_double),
                ("t_launch", C.c_double), ("t_done", C.c_double), ("batch_size", C.c_int)]


class rt_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_ulonglong), ("completed", C.c_ulonglong), ("failed", C.c_ulonglong),
                ("batches", C.c_ulonglong), ("pool_bytes", C.c_size_t), ("pool_in_use", C.c_size_t),
                ("pool_peak", C.c_size_t), ("queued", C.c_int), ("running", C.c_int)]


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = range(4)

_lib = None


def lib():
    """Load librtvol.so.  Raises ImportError when it has not been built: there
    is no fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1211_5595_amd.build` "
                              "(or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        i64p, vp, szp = C.POINTER(C.c_int64), C.c_void_p, C.POINTER(C.c_size_t)
        dp = C.POINTER(C.c_double)
        sigs = {
            "rt_volume_bytes": [i64p, C.c_int, C.c_int, C.c_int, szp],
            "rt_create_volume": [vp, C.c_int, i64p, dp, C.c_int, C.c_int, C.c_int, vp, C.c_size_t, vp,
                                 C.POINTER(vp)],
            "rt_destroy_volume": [vp],
            "rt_tf_bytes": [C.c_int, szp],
            "rt_set_transfer_function": [C.POINTER(vp), C.POINTER(C.c_float), C.c_int, C.c_double, C.c_double, vp,
                                         C.c_size_t, vp],
            "rt_destroy_tf": [vp],
            "rt_render": [vp, i64p, dp, vp, C.POINTER(rt_camera), C.c_int, C.c_int, C.c_double, C.c_double,
                          C.POINTER(C.c_float), vp, C.POINTER(rt_render_opts), vp],
            "rt_batch_workspace_bytes": [C.c_int, szp],
            "rt_render_batch": [C.POINTER(rt_render_job), C.c_int, vp, C.c_size_t, vp, C.POINTER(rt_render_opts),
                                vp],
            "rt_batch_plan_create": [C.c_int, C.c_int, C.c_int, vp, C.c_size_t, C.POINTER(rt_render_opts),
                                     C.POINTER(vp)],
            "rt_batch_plan_launch": [vp, C.POINTER(rt_render_job), C.c_int, vp, vp],
            "rt_batch_plan_destroy": [vp],
            "rt_render_batch_noalloc": [C.POINTER(rt_render_job), C.c_int, vp, C.POINTER(rt_render_opts), vp],
            "rt_server_arena_bytes": [C.c_int, C.c_int, C.c_size_t, szp],
            "rt_server_create": [C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(rt_render_opts), vp, C.c_size_t,
                                 C.c_size_t, C.POINTER(vp)],
            "rt_server_submit": [vp, C.POINTER(rt_request), C.POINTER(C.c_uint64)],
            "rt_server_wait": [vp, C.c_uint64, C.c_double, C.POINTER(rt_request_info)],
            "rt_server_release": [vp, C.c_uint64],
            "rt_server_get_stats": [vp, C.POINTER(rt_server_stats)],
            "rt_server_destroy": [vp],
        }
        for name, argt in sigs.items():
            f = getattr(L, name)
            f.argtypes = argt
            f.restype = C.c_int
        for name in ("rt_status_string",):
            getattr(L, name).restype = C.c_char_p
            getattr(L, name).argtypes = [C.c_int]
        L.rt_last_error.restype = C.c_char_p
        L.rt_last_error.argtypes = []
        L.rt_version.restype = C.c_char_p
        L.rt_batch_latency_pixels.restype = C.c_longlong
        L.rt_batch_latency_pixels.argtypes = []
        _lib = L
    return _lib


def _check(status: int, what: str):
    if status != 0:
        msg = lib().rt_last_error().decode(errors="replace")
        raise _ERRORS.get(status, RTError)(f"{what}: {msg}")


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _i64x3(x):
    return (C.c_int64 * 3)(*[int(v) for v in x])


def _f64x3(x):
    return (C.c_double * 3)(*[float(v) for v in x])


def make_camera(cam) -> rt_camera:
    c = rt_camera()
    c.eye[:] = [float(v) for v in cam.eye]
    c.center[:] = [float(v) for v in cam.center]
    c.up[:] = [float(v) for v in cam.up]
    c.perspective = 1 if cam.perspective else 0
    c.fovy_deg = float(cam.fovy_deg)
    c.ortho_half_height = float(cam.ortho_half_height)
    return c


def make_opts(sample_counter=None, pixel_counts=None, ray_function=COMPOSITE, iso_value=0.0, iso_high=0.0,
              tile=(0, 0), waves_per_block=0, skip_empty=False, tile_order=0,
              opacity_unit_distance=0.0, batch_form=0) -> rt_render_opts:
    o = rt_render_opts()
    o.batch_form = int(batch_form)
    o.tile_order = int(tile_order)
    o.opacity_unit_distance = float(opacity_unit_distance)
    o.skip_empty = 1 if skip_empty else 0
    o.sample_counter = sample_counter.data_ptr() if sample_counter is not None else None
    o.pixel_counts = pixel_counts.data_ptr() if pixel_counts is not None else None
    o.ray_function = int(ray_function)
    o.iso_value, o.iso_high = float(iso_value), float(iso_high)
    o.tile_w, o.tile_h = int(tile[0]), int(tile[1])
    o.waves_per_block = int(waves_per_block)
    return o


# ---------------------------------------------------------------------------
# C-named entry points (marshalling only)
# ---------------------------------------------------------------------------
def rt_volume_bytes(dims, storage: int, layout: int = LAYOUT_CELLS, brick: int = 0) -> int:
    n = C.c_size_t()
    _check(lib().rt_volume_bytes(_i64x3(dims), int(storage), int(layout), int(brick), C.byref(n)), "rt_volume_bytes")
    return n.value


def rt_create_volume(src_ptr: int, src_dtype: int, dims, spacing, storage: int, layout: int, brick: int,
                     dev_buf_ptr: int, dev_buf_bytes: int, stream=None) -> int:
    h = C.c_void_p()
    _check(lib().rt_create_volume(C.c_void_p(src_ptr), int(src_dtype), _i64x3(dims), _f64x3(spacing), int(storage),
                                  int(layout), int(brick), C.c_void_p(dev_buf_ptr), int(dev_buf_bytes),
                                  _stream_ptr(stream), C.byref(h)), "rt_create_volume")
    return h.value


def rt_destroy_volume(h: int):
    _check(lib().rt_destroy_volume(C.c_void_p(h)), "rt_destroy_volume")


def rt_tf_bytes(K: int) -> int:
    n = C.c_size_t()
    _check(lib().rt_tf_bytes(int(K), C.byref(n)), "rt_tf_bytes")
    return n.value


def rt_set_transfer_function(handle: Optional[int], rgba: np.ndarray, vmin: float, vmax: float, dev_buf_ptr: int,
                             dev_buf_bytes: int, stream=None) -> int:
    t = np.ascontiguousarray(rgba, dtype=np.float32)
    if t.ndim != 2 or t.shape[1] != 4:
        raise InvalidArgument("transfer function table must be K x 4")
    h = C.c_void_p(handle)
    _check(lib().rt_set_transfer_function(C.byref(h), t.ctypes.data_as(C.POINTER(C.c_float)), int(t.shape[0]),
                                          float(vmin), float(vmax), C.c_void_p(dev_buf_ptr), int(dev_buf_bytes),
                                          _stream_ptr(stream)), "rt_set_transfer_function")
    return h.value


def rt_destroy_tf(h: int):
    _check(lib().rt_destroy_tf(C.c_void_p(h)), "rt_destroy_tf")


def rt_render(vol_h: int, dims, spacing, tf_h: int, camera, width: int, height: int, step_vox: float,
              alpha_cutoff: float, bg_rgba, out_ptr: int, opts: Optional[rt_render_opts] = None, stream=None):
    bg = (C.c_float * 4)(*[float(x) for x in bg_rgba]) if bg_rgba is not None else None
    cam = make_camera(camera) if not isinstance(camera, rt_camera) else camera
    _check(lib().rt_render(C.c_void_p(vol_h), _i64x3(dims), _f64x3(spacing) if spacing is not None else None,
                           C.c_void_p(tf_h), C.byref(cam), int(width), int(height), float(step_vox),
                           float(alpha_cutoff), bg, C.c_void_p(out_ptr), C.byref(opts) if opts is not None else None,
                           _stream_ptr(stream)), "rt_render")


def rt_batch_workspace_bytes(max_jobs: int) -> int:
    n = C.c_size_t()
    _check(lib().rt_batch_workspace_bytes(int(max_jobs), C.byref(n)), "rt_batch_workspace_bytes")
    return n.value


def rt_render_batch(jobs, ws_ptr: int, ws_bytes: int, counter_ptr: Optional[int] = None,
                    opts: Optional[rt_render_opts] = None, stream=None):
    arr = (rt_render_job * len(jobs))(*jobs)
    _check(lib().rt_render_batch(arr, len(jobs), C.c_void_p(ws_ptr), int(ws_bytes), C.c_void_p(counter_ptr),
                                 C.byref(opts) if opts is not None else None, _stream_ptr(stream)), "rt_render_batch")


def rt_render_batch_noalloc(jobs, counter_ptr: Optional[int] = None, opts: Optional[rt_render_opts] = None,
                            stream=None):
    arr = (rt_render_job * len(jobs))(*jobs)
    _check(lib().rt_render_batch_noalloc(arr, len(jobs), C.c_void_p(counter_ptr),
                                         C.byref(opts) if opts is not None else None, _stream_ptr(stream)),
           "rt_render_batch_noalloc")


def rt_batch_plan_create(max_jobs: int, storage: int, layout: int, ws_ptr: int, ws_bytes: int,
                         opts: Optional[rt_render_opts] = None) -> int:
    h = C.c_void_p()
    _check(lib().rt_batch_plan_create(int(max_jobs), int(storage), int(layout), C.c_void_p(ws_ptr), int(ws_bytes),
                                      C.byref(opts) if opts is not None else None, C.byref(h)), "rt_batch_plan_create")
    return h.value


def rt_batch_plan_launch(plan_h: int, jobs, counter_ptr: Optional[int] = None, stream=None):
    arr = (rt_render_job * len(jobs))(*jobs)
    _check(lib().rt_batch_plan_launch(C.c_void_p(plan_h), arr, len(jobs), C.c_void_p(counter_ptr),
                                      _stream_ptr(stream)), "rt_batch_plan_launch")


def rt_batch_latency_pixels() -> int:
    """Pixels up to which a plan (batch_form 0) takes the latency form."""
    return int(lib().rt_batch_latency_pixels())


def rt_batch_plan_destroy(plan_h: int):
    _check(lib().rt_batch_plan_destroy(C.c_void_p(plan_h)), "rt_batch_plan_destroy")


def rt_server_arena_bytes(n_streams: int, max_batch: int, image_pool_bytes: int) -> int:
    b = C.c_size_t()
    _check(lib().rt_server_arena_bytes(n_streams, max_batch, image_pool_bytes, C.byref(b)), "rt_server_arena_bytes")
    return b.value


def rt_server_create(n_streams: int, max_batch: int, storage: int, layout: int, opts, arena_ptr: int,
                     arena_bytes: int, image_pool_bytes: int) -> int:
    h = C.c_void_p()
    _check(lib().rt_server_create(n_streams, max_batch, storage, layout, C.byref(opts) if opts is not None else None,
                                  C.c_void_p(arena_ptr), arena_bytes, image_pool_bytes, C.byref(h)),
           "rt_server_create")
    return h.value


def rt_server_submit(server_h: int, req: rt_request) -> int:
    t = C.c_uint64()
    _check(lib().rt_server_submit(C.c_void_p(server_h), C.byref(req), C.byref(t)), "rt_server_submit")
    return t.value


def rt_server_wait(server_h: int, ticket: int, timeout_s: float = -1.0) -> rt_request_info:
    info = rt_request_info()
    _check(lib().rt_server_wait(C.c_void_p(server_h), ticket, timeout_s, C.byref(info)), "rt_server_wait")
    return info


def rt_server_release(server_h: int, ticket: int):
    _check(lib().rt_server_release(C.c_void_p(server_h), ticket), "rt_server_release")


def rt_server_get_stats(server_h: int) -> rt_server_stats:
    st = rt_server_stats()
    _check(lib().rt_server_get_stats(C.c_void_p(server_h), C.byref(st)), "rt_server_get_stats")
    return st


def rt_server_destroy(server_h: int):
    _check(lib().rt_server_destroy(C.c_void_p(server_h)), "rt_server_destroy")


# ---------------------------------------------------------------------------
# handle classes owning their torch buffers
# ---------------------------------------------------------------------------
class Volume:
    """A volume resident in device memory in the raycaster's storage layout.

    ``values``: numpy array or CUDA tensor, C-order [z][y][x] of uint8,
    uint16, float16 or float32.  ``storage``: one of U8, U16, F16, F32
    (``layout`` LAYOUT_CELLS or LAYOUT_LINEAR; LAYOUT_POLY for U8/U16;
    LAYOUT_QUADS for U16 and U12, which also take LAYOUT_CELLS) or
    U8_BRICKSCALED (``brick`` 8/16/32, ``layout`` LAYOUT_CELLS or
    LAYOUT_BRICKS).  With ``stream`` given, the conversion runs there after
    the work already queued on the current stream (which produced the
    source)."""

    def __init__(self, values, spacing: Sequence[float], storage: Optional[int] = None, brick: int = 0,
                 stream=None, device="cuda", layout: int = LAYOUT_CELLS):
        torch = _torch()
        if isinstance(values, np.ndarray):
            arr = np.ascontiguousarray(values)
            src_dtype = _DTYPE_CODE.get(arr.dtype)
            if src_dtype is None:
                raise InvalidArgument(f"unsupported source dtype {arr.dtype}")
            view = arr.view(np.int16) if arr.dtype == np.uint16 else arr
            src = torch.from_numpy(view).to(device)
        else:
            src = values.contiguous()
            tmap = {torch.uint8: U8, torch.int16: U16, torch.float16: F16, torch.float32: F32}
            if getattr(torch, "uint16", None) is not None:
                tmap[torch.uint16] = U16
            src_dtype = tmap.get(src.dtype)
            if src_dtype is None:
                raise InvalidArgument(f"unsupported source dtype {src.dtype}")
        nz, ny, nx = src.shape
        self.dims = (nx, ny, nz)
        self.spacing = tuple(float(s) for s in spacing)
        self.storage = src_dtype if storage is None else int(storage)
        self.brick = int(brick)
        self.layout = int(layout)
        self.nbytes = rt_volume_bytes(self.dims, self.storage, self.layout, self.brick)
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=src.device)
        if stream is not None:
            stream.wait_stream(torch.cuda.current_stream(src.device))   # the source copy / producer
            self.buf.record_stream(stream)
            src.record_stream(stream)
        self.handle = rt_create_volume(src.data_ptr(), src_dtype, self.dims, self.spacing, self.storage, self.layout,
                                       self.brick, self.buf.data_ptr(), self.nbytes, stream)
        self._src = src  # kept until the relayout on the stream has consumed it
        if stream is None:
            torch.cuda.current_stream(src.device).synchronize()
            self._src = None

    def close(self):
        if getattr(self, "handle", None):
            rt_destroy_volume(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TransferFunction:
    """K x 4 RGBA table over [vmin, vmax], copied into a device buffer."""

    def __init__(self, rgba: np.ndarray, vmin: float, vmax: float, stream=None, device="cuda"):
        torch = _torch()
        t = np.ascontiguousarray(rgba, dtype=np.float32)
        self.K = int(t.shape[0])
        self.vmin, self.vmax = float(vmin), float(vmax)
        self.nbytes = rt_tf_bytes(self.K)
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        if stream is not None:
            self.buf.record_stream(stream)
        self.handle = rt_set_transfer_function(None, t, vmin, vmax, self.buf.data_ptr(), self.nbytes, stream)
        self.table = t

    def update(self, rgba: np.ndarray, vmin: Optional[float] = None, vmax: Optional[float] = None, stream=None):
        t = np.ascontiguousarray(rgba, dtype=np.float32)
        self.vmin = self.vmin if vmin is None else float(vmin)
        self.vmax = self.vmax if vmax is None else float(vmax)
        self.handle = rt_set_transfer_function(self.handle, t, self.vmin, self.vmax, 0, 0, stream)
        self.table = t
        self.K = int(t.shape[0])

    def close(self):
        if getattr(self, "handle", None):
            rt_destroy_tf(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def render(volume: Volume, tf: TransferFunction, camera, width: int, height: int, step_vox: float = 0.5,
           alpha_cutoff: float = 0.99, bg=(0.0, 0.0, 0.0, 0.0), out=None, pixel_counts=None, sample_counter=None,
           spacing=None, tile=(0, 0), waves_per_block=0, stream=None, ray_function=COMPOSITE, iso_value=0.0,
           iso_high=0.0, skip_empty=False, tile_order=0, opacity_unit_distance=0.0):
    """Render one view; returns the float32 [H][W][4] device image."""
    torch = _torch()
    if out is None:
        out = torch.empty((height, width, 4), dtype=torch.float32, device=volume.buf.device)
    opts = make_opts(sample_counter, pixel_counts, ray_function, iso_value, iso_high, tile=tile,
                     waves_per_block=waves_per_block, skip_empty=skip_empty, tile_order=tile_order,
                     opacity_unit_distance=opacity_unit_distance)
    rt_render(volume.handle, volume.dims, spacing, tf.handle, camera, width, height, step_vox, alpha_cutoff, bg,
              out.data_ptr(), opts, stream)
    return out


class Job:
    """One view of a batch."""

    def __init__(self, volume: Volume, tf: TransferFunction, camera, width: int, height: int,
                 step_vox: float = 0.5, alpha_cutoff: float = 0.99, bg=(0.0, 0.0, 0.0, 0.0), out=None,
                 pixel_counts=None, ray_function: int = COMPOSITE, iso_value: float = 0.0, iso_high: float = 0.0,
                 skip_empty: bool = False, opacity_unit_distance: float = 0.0):
        torch = _torch()
        self.volume, self.tf, self.camera = volume, tf, camera
        self.ray_function, self.iso_value, self.iso_high = int(ray_function), float(iso_value), float(iso_high)
        self.skip_empty = bool(skip_empty)
        self.opacity_unit_distance = float(opacity_unit_distance)
        self.width, self.height = int(width), int(height)
        self.step_vox, self.alpha_cutoff, self.bg = float(step_vox), float(alpha_cutoff), tuple(bg)
        self.out = out if out is not None else torch.empty((height, width, 4), dtype=torch.float32,
                                                           device=volume.buf.device)
        self.pixel_counts = pixel_counts

    def struct(self) -> rt_render_job:
        j = rt_render_job()
        j.volume, j.tf = self.volume.handle, self.tf.handle
        j.camera = make_camera(self.camera)
        j.width, j.height = self.width, self.height
        j.step_vox, j.alpha_cutoff = self.step_vox, self.alpha_cutoff
        j.bg_rgba[:] = [float(x) for x in self.bg]
        j.out_dev = self.out.data_ptr()
        j.pixel_counts = self.pixel_counts.data_ptr() if self.pixel_counts is not None else None
        j.ray_function, j.iso_value, j.iso_high = self.ray_function, self.iso_value, self.iso_high
        j.skip_empty = 1 if self.skip_empty else 0
        j.opacity_unit_distance = self.opacity_unit_distance
        return j


class _Workspace:
    def __init__(self, max_jobs: int, device="cuda"):
        torch = _torch()
        self.max_jobs = max_jobs
        self.nbytes = rt_batch_workspace_bytes(max_jobs)
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device)


_ws_cache = {}


def render_batch(jobs: Sequence[Job], sample_counter=None, workspace=None, tile=(0, 0), waves_per_block=0,
                 stream=None, tile_order=0):
    """Render all jobs in one persistent launch (job table copied per call).
    Without ``workspace``, one is kept per device, batch size and stream: calls
    on one stream reuse it in stream order, and calls on different streams
    never share one (a job table copied for one stream could otherwise land
    while another stream's launch still reads the same memory)."""
    n = len(jobs)
    dev = jobs[0].out.device
    if workspace is None:
        key = (str(dev), n, _stream_ptr(stream).value)
        workspace = _ws_cache.get(key)
        if workspace is None:
            workspace = _ws_cache[key] = _Workspace(n, dev)
    opts = make_opts(None, None, COMPOSITE, tile=tile, waves_per_block=waves_per_block, tile_order=tile_order)
    rt_render_batch([j.struct() for j in jobs], workspace.buf.data_ptr(), workspace.nbytes,
                    sample_counter.data_ptr() if sample_counter is not None else None, opts, stream)
    return [j.out for j in jobs]


class BatchPlan:
    """The persistent batched launch captured once in a HIP graph, and its
    latency form for small batches (batch_form: 0 by size, 1 persistent
    always, 2 latency form always)."""

    def __init__(self, max_jobs: int, storage: int, tile=(0, 0), waves_per_block=0, device="cuda",
                 layout: int = LAYOUT_CELLS, skip_empty: bool = False, tile_order: int = 0, batch_form: int = 0):
        self.ws = _Workspace(max_jobs, device)
        self.handle = rt_batch_plan_create(max_jobs, storage, layout, self.ws.buf.data_ptr(), self.ws.nbytes,
                                           make_opts(tile=tile, waves_per_block=waves_per_block,
                                                     skip_empty=skip_empty, tile_order=tile_order,
                                                     batch_form=batch_form))

    def launch(self, jobs: Sequence[Job], sample_counter=None, stream=None):
        rt_batch_plan_launch(self.handle, [j.struct() for j in jobs],
                             sample_counter.data_ptr() if sample_counter is not None else None, stream)
        return [j.out for j in jobs]

    def close(self):
        if getattr(self, "handle", None):
            rt_batch_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
