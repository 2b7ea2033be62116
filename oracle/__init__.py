"""FP64 CPU reference raycaster -- TEST INFRASTRUCTURE ONLY.

The correctness oracle for the GPU raycaster.  Only ``tests/``, the package
smoke check (``__graft_entry__.smoke``) and the benchmark's CPU-baseline leg
may import this module; the product path never does.  It shares no code with
the GPU library: it is a plain C library (``oracle.c``, its own header
``oracle.h``) loaded through ctypes, plus numpy marshalling.

What it computes follows arXiv:1211.5595 -- Section 4.1 (one viewing ray per
pixel, intersected with the volume, evenly spaced samples; three ray-casting
steps), Section 3.2 (trilinear resampling), Sections 2.6 and 6 (colour and
opacity transfer functions) and Section 4.2 eqs. (1)-(5) (compositing).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import sys
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

COMPOSITE, MIP, XRAY, AVERAGE, ISO, THRESHOLD = range(6)
TRACE_FIELDS = ("s", "weight", "qx", "qy", "qz", "value", "r", "g", "b", "a", "alpha",
                "Cr", "Cg", "Cb", "T", "count")


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (binary64, no FP contraction, OpenMP)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    src = os.path.join(_HERE, "oracle.c")
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter", src, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Camera(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("center", C.c_double * 3), ("up", C.c_double * 3),
                ("perspective", C.c_int), ("fovy_deg", C.c_double), ("ortho_half_height", C.c_double)]


class _Volume(C.Structure):
    _fields_ = [("dims", C.c_int64 * 3), ("spacing", C.c_double * 3), ("field", C.POINTER(C.c_double)),
                ("brick", C.c_int), ("brick_lo", C.POINTER(C.c_float)),
                ("brick_scale", C.POINTER(C.c_float)), ("codes", C.POINTER(C.c_uint8))]


class _TF(C.Structure):
    _fields_ = [("rgba", C.POINTER(C.c_float)), ("K", C.c_int), ("vmin", C.c_double), ("vmax", C.c_double)]


class _Params(C.Structure):
    _fields_ = [("width", C.c_int), ("height", C.c_int), ("step_vox", C.c_double), ("cutoff", C.c_double),
                ("bg", C.c_double * 4), ("ray_function", C.c_int), ("iso_value", C.c_double),
                ("iso_high", C.c_double), ("tie_delta", C.c_double), ("opacity_unit", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp, ip, fp, u8p = C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_float), C.POINTER(C.c_uint8)
        L.orc_camera_frame.argtypes = [C.POINTER(_Camera), dp, dp, dp]
        L.orc_pixel_ray.argtypes = [C.POINTER(_Camera), C.c_int, C.c_int, C.c_int, C.c_int, dp, dp]
        L.orc_box_clip.argtypes = [dp, dp, dp, dp, dp]
        L.orc_lattice.argtypes = [C.c_double, C.c_double, ip, dp]
        L.orc_lattice.restype = C.c_int64
        L.orc_trilinear.argtypes = [C.POINTER(_Volume), dp]
        L.orc_trilinear.restype = C.c_double
        L.orc_classify.argtypes = [C.POINTER(_TF), C.c_double, dp]
        L.orc_classify.restype = None
        L.orc_render.argtypes = [C.POINTER(_Volume), C.POINTER(_TF), C.POINTER(_Camera), C.POINTER(_Params),
                                 ip, C.c_int64, dp, ip, dp, dp, u8p, C.c_int]
        L.orc_trace_ray.argtypes = [C.POINTER(_Volume), C.POINTER(_TF), C.POINTER(_Camera), C.POINTER(_Params),
                                    C.c_int, C.c_int, dp, C.c_int64]
        L.orc_trace_ray.restype = C.c_int64
        L.orc_u8_brick_count.argtypes = [ip, C.c_int, ip]
        L.orc_u8_brick_count.restype = C.c_int64
        L.orc_encode_u8_bricks.argtypes = [dp, ip, C.c_int, fp, fp, u8p]
        L.orc_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _camera(cam) -> _Camera:
    c = _Camera()
    c.eye[:] = [float(x) for x in cam.eye]
    c.center[:] = [float(x) for x in cam.center]
    c.up[:] = [float(x) for x in cam.up]
    c.perspective = 1 if cam.perspective else 0
    c.fovy_deg = float(cam.fovy_deg)
    c.ortho_half_height = float(cam.ortho_half_height)
    return c


class Volume:
    """A node-centred scalar volume as the oracle sees it: either a plain
    field (``values``: array [z][y][x] of node values, converted exactly to
    float64) or 8-bit per-brick codes (``from_u8_bricks``)."""

    def __init__(self, values: Optional[np.ndarray], spacing: Sequence[float], dims=None):
        self._keep = []
        self.s = _Volume()
        if values is not None:
            f = np.ascontiguousarray(values, dtype=np.float64)
            nz, ny, nx = f.shape
            self.dims = (nx, ny, nz)
            self.field = f
            self.s.field = _ptr(f, C.c_double)
            self._keep.append(f)
        else:
            self.dims = tuple(int(x) for x in dims)
            self.field = None
        self.spacing = tuple(float(x) for x in spacing)
        self.s.dims[:] = list(self.dims)
        self.s.spacing[:] = list(self.spacing)

    @classmethod
    def from_u8_bricks(cls, values: np.ndarray, spacing, B: int):
        """Encode ``values`` with the 8-bit per-brick scaled code (brick size B)
        and return the decoded-on-the-fly volume plus (lo, scale, codes)."""
        lo, scale, codes = encode_u8_bricks(values, B)
        nz, ny, nx = values.shape
        v = cls(None, spacing, dims=(nx, ny, nz))
        v.s.brick = B
        v.brick = B
        v.lo, v.scale, v.codes = lo, scale, codes
        v.s.brick_lo = _ptr(lo, C.c_float)
        v.s.brick_scale = _ptr(scale, C.c_float)
        v.s.codes = _ptr(codes, C.c_uint8)
        v._keep += [lo, scale, codes]
        return v


class TF:
    def __init__(self, rgba: np.ndarray, vmin: float, vmax: float):
        t = np.ascontiguousarray(rgba, dtype=np.float32)
        assert t.ndim == 2 and t.shape[1] == 4
        self.rgba = t
        self.s = _TF(_ptr(t, C.c_float), t.shape[0], float(vmin), float(vmax))


def _params(width, height, step_vox, cutoff, bg=(0, 0, 0, 0), ray_function=COMPOSITE, iso_value=0.0,
            iso_high=0.0, tie_delta=0.0, opacity_unit=0.0) -> _Params:
    p = _Params()
    p.width, p.height = int(width), int(height)
    p.step_vox, p.cutoff = float(step_vox), float(cutoff)
    p.bg[:] = [float(x) for x in bg]
    p.ray_function = int(ray_function)
    p.iso_value, p.iso_high = float(iso_value), float(iso_high)
    p.tie_delta = float(tie_delta)
    p.opacity_unit = float(opacity_unit)
    return p


class RenderResult:
    def __init__(self, image, counts, band_lo, band_hi, tie):
        self.image, self.counts, self.band_lo, self.band_hi, self.tie = image, counts, band_lo, band_hi, tie


def render(vol: Volume, tf: TF, cam, width: int, height: int, step_vox: float, cutoff: float,
           bg=(0.0, 0.0, 0.0, 0.0), pixels: Optional[np.ndarray] = None, tie_delta: float = 0.0,
           ray_function: int = COMPOSITE, iso_value: float = 0.0, iso_high: float = 0.0,
           nthreads: int = 0, want_band: bool = False, opacity_unit: float = 0.0) -> RenderResult:
    """Render the whole image (``pixels`` None -> float64 [H][W][4]) or the
    listed pixel ids (j*W + i -> float64 [n][4]).  opacity_unit > 0 applies
    the opacity correction to that unit distance (compositing, thresholding)."""
    L = lib()
    prm = _params(width, height, step_vox, cutoff, bg, ray_function, iso_value, iso_high, tie_delta, opacity_unit)
    camc = _camera(cam)
    if pixels is None:
        n = width * height
        pix_ptr = None
    else:
        px = np.ascontiguousarray(pixels, dtype=np.int64)
        n = px.size
        pix_ptr = _ptr(px, C.c_int64)
    out = np.zeros((n, 4), dtype=np.float64)
    counts = np.zeros(n, dtype=np.int64)
    tie = np.zeros(n, dtype=np.uint8)
    lo = np.zeros((n, 4), dtype=np.float64) if want_band else None
    hi = np.zeros((n, 4), dtype=np.float64) if want_band else None
    rc = L.orc_render(C.byref(vol.s), C.byref(tf.s), C.byref(camc), C.byref(prm), pix_ptr, n,
                      _ptr(out, C.c_double), _ptr(counts, C.c_int64),
                      _ptr(lo, C.c_double) if want_band else None, _ptr(hi, C.c_double) if want_band else None,
                      _ptr(tie, C.c_uint8), int(nthreads))
    if rc != 0:
        raise ValueError("oracle: invalid render arguments")
    if pixels is None:
        out = out.reshape(height, width, 4)
        counts = counts.reshape(height, width)
        tie = tie.reshape(height, width)
        if want_band:
            lo, hi = lo.reshape(height, width, 4), hi.reshape(height, width, 4)
    return RenderResult(out, counts, lo, hi, tie)


def trace_ray(vol: Volume, tf: TF, cam, width, height, i, j, step_vox, cutoff, bg=(0, 0, 0, 0),
              max_rec: int = 100000) -> np.ndarray:
    """Per-sample records of one pixel's ray: structured float64 array with
    fields ``TRACE_FIELDS``."""
    prm = _params(width, height, step_vox, cutoff, bg)
    rec = np.zeros((max_rec, 16), dtype=np.float64)
    n = lib().orc_trace_ray(C.byref(vol.s), C.byref(tf.s), C.byref(_camera(cam)), C.byref(prm), int(i), int(j),
                            _ptr(rec, C.c_double), max_rec)
    if n < 0:
        raise ValueError("oracle: invalid trace arguments")
    return rec[:n]


def camera_frame(cam):
    w, u, v = (np.zeros(3) for _ in range(3))
    rc = lib().orc_camera_frame(C.byref(_camera(cam)), _ptr(w, C.c_double), _ptr(u, C.c_double),
                                _ptr(v, C.c_double))
    if rc != 0:
        raise ValueError("oracle: invalid camera")
    return w, u, v


def pixel_ray(cam, W, H, i, j):
    o, d = np.zeros(3), np.zeros(3)
    rc = lib().orc_pixel_ray(C.byref(_camera(cam)), int(W), int(H), int(i), int(j), _ptr(o, C.c_double),
                             _ptr(d, C.c_double))
    if rc != 0:
        raise ValueError("oracle: invalid camera")
    return o, d


def box_clip(o, d, hi):
    o, d, hi = (np.ascontiguousarray(x, dtype=np.float64) for x in (o, d, hi))
    tn, tf = C.c_double(), C.c_double()
    hit = lib().orc_box_clip(_ptr(o, C.c_double), _ptr(d, C.c_double), _ptr(hi, C.c_double), C.byref(tn),
                             C.byref(tf))
    return bool(hit), tn.value, tf.value


def lattice(L: float, dt: float):
    m, r = C.c_int64(), C.c_double()
    n = lib().orc_lattice(float(L), float(dt), C.byref(m), C.byref(r))
    return int(n), int(m.value), float(r.value)


def trilinear(vol: Volume, q) -> float:
    qa = np.ascontiguousarray(q, dtype=np.float64)
    return float(lib().orc_trilinear(C.byref(vol.s), _ptr(qa, C.c_double)))


def classify(tf: TF, value: float) -> np.ndarray:
    out = np.zeros(4)
    lib().orc_classify(C.byref(tf.s), float(value), _ptr(out, C.c_double))
    return out


def u8_brick_count(dims, B):
    d = np.array(dims, dtype=np.int64)
    nb = np.zeros(3, dtype=np.int64)
    total = lib().orc_u8_brick_count(_ptr(d, C.c_int64), int(B), _ptr(nb, C.c_int64))
    return int(total), tuple(int(x) for x in nb)


def encode_u8_bricks(values: np.ndarray, B: int):
    """Per-brick scaled 8-bit code of a [z][y][x] volume: returns
    (lo float32[nb], scale float32[nb], codes uint8[nb][(B+1)^3])."""
    f = np.ascontiguousarray(values, dtype=np.float64)
    nz, ny, nx = f.shape
    d = np.array([nx, ny, nz], dtype=np.int64)
    total, nb = u8_brick_count((nx, ny, nz), B)
    lo = np.zeros(total, dtype=np.float32)
    sc = np.zeros(total, dtype=np.float32)
    codes = np.zeros((total, (B + 1) ** 3), dtype=np.uint8)
    rc = lib().orc_encode_u8_bricks(_ptr(f, C.c_double), _ptr(d, C.c_int64), int(B), _ptr(lo, C.c_float),
                                    _ptr(sc, C.c_float), _ptr(codes, C.c_uint8))
    if rc != 0:
        raise ValueError("oracle: invalid encode arguments")
    return lo, sc, codes


def max_threads() -> int:
    return int(lib().orc_max_threads())


if __name__ == "__main__":
    print(build(), file=sys.stderr)
