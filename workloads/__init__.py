"""Seeded synthetic workloads for the raycaster: phantoms, transfer functions,
cameras and request streams.

This module is shared by the FP64 oracle (``oracle/``), the tests and the
benchmark.  It holds no step of the rendering method itself: it only draws
inputs (volumes, RGBA tables, camera poses, arrival times) from seeded
``numpy.random.default_rng`` streams.

The paper's data are 50-100 private brain MRI volumes (Section 4.4); none are
available, so brain-like phantoms stand in for them.  MRI slices come with a
slice thickness and gaps (Section 1), which is why every phantom carries an
anisotropic voxel spacing.

Conventions (shared with both implementations):
  * a volume array is C-order ``[z][y][x]`` (x fastest); ``dims = (nx, ny, nz)``;
  * voxel ``(i, j, k)`` sits at physical position ``(i*sx, j*sy, k*sz)`` mm;
  * a transfer-function table is ``float32[K][4]`` RGBA in ``[0, 1]``, entry
    ``j`` belonging to value ``vmin + j*(vmax-vmin)/(K-1)``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, NamedTuple, Sequence, Tuple

import numpy as np

__all__ = [
    "Camera", "VolumeSpec", "TFSpec",
    "phantom_small", "phantom_brain", "random_tf", "tf_from_points",
    "box_center", "bounding_radius", "ortho_camera_small", "orbit_cameras",
    "random_camera", "random_views", "poisson_requests",
    "CONFIG_SMALL", "CONFIG_BRAIN", "BATCH_SIZES",
]


class Camera(NamedTuple):
    """Look-at camera (plain data).  ``perspective`` selects pinhole (with
    ``fovy_deg``, the full vertical field of view) or orthographic (with
    ``ortho_half_height`` in mm)."""
    eye: Tuple[float, float, float]
    center: Tuple[float, float, float]
    up: Tuple[float, float, float]
    perspective: bool
    fovy_deg: float = 0.0
    ortho_half_height: float = 0.0


@dataclasses.dataclass(frozen=True)
class VolumeSpec:
    dims: Tuple[int, int, int]          # (nx, ny, nz)
    spacing: Tuple[float, float, float]  # mm
    dtype: str                           # "u8" | "u16"
    seed: int


@dataclasses.dataclass(frozen=True)
class TFSpec:
    K: int
    vmin: float
    vmax: float
    alpha_max: float
    seed: int


# The two single-volume workloads (small correctness case, brain-sized case).
CONFIG_SMALL = dict(volume=VolumeSpec((64, 64, 32), (1.0, 1.0, 2.0), "u8", 1),
                    tf=TFSpec(256, 0.0, 255.0, 1.0, 2),
                    width=128, height=128, step_vox=0.5, cutoff=0.99)
CONFIG_BRAIN = dict(volume=VolumeSpec((256, 256, 160), (0.9, 0.9, 1.2), "u16", 11),
                    tf=TFSpec(4096, 0.0, 4095.0, 0.05, 12),
                    width=512, height=512, step_vox=0.5, cutoff=0.99, n_views=36)
# Volume sizes of the uneven-batch workload.
BATCH_SIZES = [(128, 128, 64), (192, 192, 96), (256, 256, 160), (512, 512, 256)]


# --------------------------------------------------------------------------
# geometry helpers (inputs only: box centre and bounding sphere of a volume)
# --------------------------------------------------------------------------
def box_center(dims: Sequence[int], spacing: Sequence[float]) -> np.ndarray:
    return np.array([(n - 1) * s / 2.0 for n, s in zip(dims, spacing)], dtype=np.float64)


def bounding_radius(dims: Sequence[int], spacing: Sequence[float]) -> float:
    half = np.array([(n - 1) * s / 2.0 for n, s in zip(dims, spacing)])
    return float(np.sqrt((half ** 2).sum()))


def _node_coords(dims, spacing, z_index):
    """Physical (x, y) grids of one z-slice and its z coordinate, relative to
    the box centre."""
    nx, ny, nz = dims
    c = box_center(dims, spacing)
    x = np.arange(nx, dtype=np.float64) * spacing[0] - c[0]
    y = np.arange(ny, dtype=np.float64) * spacing[1] - c[1]
    z = z_index * spacing[2] - c[2]
    return x[None, :], y[:, None], z


def _inside_ellipsoid(x, y, z, centre, semi):
    return (((x - centre[0]) / semi[0]) ** 2 + ((y - centre[1]) / semi[1]) ** 2
            + ((z - centre[2]) / semi[2]) ** 2) <= 1.0


def _paint(dims, spacing, shapes, background: float) -> np.ndarray:
    """Paint shapes (list of (centre, semi_axes, value)) in order, later shapes
    over earlier ones; "inside" is tested at voxel nodes.  Returns float64
    ``[z][y][x]``.  Each shape is evaluated only on the bounding box of its
    cross-section with the slice (plus one node of margin); nodes outside it
    are outside the ellipsoid, so the result equals a full evaluation."""
    nx, ny, nz = dims
    c = box_center(dims, spacing)
    out = np.full((nz, ny, nx), background, dtype=np.float64)
    for k in range(nz):
        x, y, z = _node_coords(dims, spacing, k)
        sl = out[k]
        for centre, semi, value in shapes:
            dz = (z - centre[2]) / semi[2]
            if abs(dz) > 1.0:
                continue
            r = math.sqrt(max(0.0, 1.0 - dz * dz))
            i0 = max(0, int(math.floor((centre[0] - semi[0] * r + c[0]) / spacing[0])) - 1)
            i1 = min(nx, int(math.ceil((centre[0] + semi[0] * r + c[0]) / spacing[0])) + 2)
            j0 = max(0, int(math.floor((centre[1] - semi[1] * r + c[1]) / spacing[1])) - 1)
            j1 = min(ny, int(math.ceil((centre[1] + semi[1] * r + c[1]) / spacing[1])) + 2)
            if i0 >= i1 or j0 >= j1:
                continue
            m = _inside_ellipsoid(x[:, i0:i1], y[j0:j1, :], z, centre, semi)
            sl[j0:j1, i0:i1][m] = value
    return out


def _uniform_in_ellipsoid(rng, semi, shrink=0.0):
    """Rejection-sample a point uniformly inside an ellipsoid centred at 0,
    with each semi-axis reduced by ``shrink`` mm."""
    a = np.maximum(np.asarray(semi, dtype=np.float64) - shrink, 1e-9)
    while True:
        p = rng.uniform(-1.0, 1.0, size=3)
        if (p ** 2).sum() <= 1.0:
            return p * a


# --------------------------------------------------------------------------
# phantoms
# --------------------------------------------------------------------------
def phantom_small(seed: int = 1, dims=(64, 64, 32), spacing=(1.0, 1.0, 2.0)) -> np.ndarray:
    """Small head phantom, uint8 ``[z][y][x]``: skull shell (200) between
    ellipsoids with semi-axes (26,30,28) and (23,27,25) mm, brain (110),
    two ventricles (40), one tumour sphere (240) of radius 5 voxels along the
    finest axis, background 0, Gaussian noise sigma 4, rounded half-to-even
    and clipped to [0, 255]."""
    rng = np.random.default_rng(seed)
    outer, inner = (26.0, 30.0, 28.0), (23.0, 27.0, 25.0)
    r_t = 5.0 * min(spacing)
    t_c = _uniform_in_ellipsoid(rng, inner, shrink=6.0)
    shapes = [
        ((0.0, 0.0, 0.0), outer, 200.0),
        ((0.0, 0.0, 0.0), inner, 110.0),
        ((5.0, 2.0, 2.0), (3.0, 8.0, 4.0), 40.0),
        ((-5.0, 2.0, 2.0), (3.0, 8.0, 4.0), 40.0),
        (tuple(t_c), (r_t, r_t, r_t), 240.0),
    ]
    vol = _paint(dims, spacing, shapes, 0.0)
    vol += rng.normal(0.0, 4.0, size=vol.shape)
    return np.clip(np.rint(vol), 0, 255).astype(np.uint8)


def phantom_small_symmetric(seed: int = 1, dims=(64, 64, 32), spacing=(1.0, 1.0, 2.0)) -> np.ndarray:
    """The small phantom without noise and with the tumour on the x = centre
    plane, so the volume is mirror-symmetric in x."""
    rng = np.random.default_rng(seed)
    t_c = _uniform_in_ellipsoid(rng, (23.0, 27.0, 25.0), shrink=6.0)
    t_c[0] = 0.0
    r_t = 5.0 * min(spacing)
    shapes = [
        ((0.0, 0.0, 0.0), (26.0, 30.0, 28.0), 200.0),
        ((0.0, 0.0, 0.0), (23.0, 27.0, 25.0), 110.0),
        ((5.0, 2.0, 2.0), (3.0, 8.0, 4.0), 40.0),
        ((-5.0, 2.0, 2.0), (3.0, 8.0, 4.0), 40.0),
        (tuple(t_c), (r_t, r_t, r_t), 240.0),
    ]
    vol = _paint(dims, spacing, shapes, 0.0)
    return np.clip(np.rint(vol), 0, 255).astype(np.uint8)


def phantom_brain(seed: int = 11, dims=(256, 256, 160), spacing=(0.9, 0.9, 1.2),
                  rician_sigma: float = 20.0) -> np.ndarray:
    """Brain-like uint16 phantom on a 12-bit range, ``[z][y][x]``.

    Nested ellipsoids with semi-axes ``f*(0.80hx, 0.95hy, 0.90hz)`` (h = box
    half-extent), each axis jittered by up to +-5 %:
        f=1.00 skin 1500, 0.95 skull 400, 0.90 CSF 900, 0.86 grey 1800,
        0.70 white 2400;
    two ventricles (900); three tumour spheres of radius U[4,15] voxels along
    the finest axis (3300) centred inside the f=0.80 ellipsoid.  Background 0.
    Rician noise: sqrt((v+n1)^2 + n2^2), n1, n2 ~ N(0, sigma^2); then rounded
    half-to-even and clipped to [0, 4095]."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    h = np.array([(n - 1) * s / 2.0 for n, s in zip(dims, spacing)])
    base = np.array([0.80, 0.95, 0.90]) * h
    shapes = []
    for f, value in ((1.00, 1500.0), (0.95, 400.0), (0.90, 900.0), (0.86, 1800.0), (0.70, 2400.0)):
        jitter = rng.uniform(0.95, 1.05, size=3)
        shapes.append(((0.0, 0.0, 0.0), tuple(f * base * jitter), value))
    vsemi = tuple(np.array([0.05, 0.14, 0.07]) * h)
    voff = np.array([0.08, 0.03, 0.06]) * h
    shapes.append(((voff[0], voff[1], voff[2]), vsemi, 900.0))
    shapes.append(((-voff[0], voff[1], voff[2]), vsemi, 900.0))
    for _ in range(3):
        r = rng.uniform(4.0, 15.0) * min(spacing)
        c = _uniform_in_ellipsoid(rng, 0.80 * base)
        shapes.append((tuple(c), (r, r, r), 3300.0))
    out = np.empty((nz, ny, nx), dtype=np.uint16)
    clean = _paint(dims, spacing, shapes, 0.0)
    for k in range(nz):  # slice-wise noise keeps temporaries small
        n1 = rng.normal(0.0, rician_sigma, size=(ny, nx))
        n2 = rng.normal(0.0, rician_sigma, size=(ny, nx))
        v = np.sqrt((clean[k] + n1) ** 2 + n2 ** 2)
        out[k] = np.clip(np.rint(v), 0, 4095).astype(np.uint16)
    return out


# --------------------------------------------------------------------------
# transfer functions
# --------------------------------------------------------------------------
def tf_from_points(K: int, positions: Sequence[float], rgba: Sequence[Sequence[float]]) -> np.ndarray:
    """Sample a piecewise-linear RGBA curve, given at normalised positions in
    [0, 1] (held constant beyond the last point), at K evenly spaced entries.
    Returns float32 [K][4]."""
    pos = np.asarray(positions, dtype=np.float64)
    val = np.asarray(rgba, dtype=np.float64)
    u = np.arange(K, dtype=np.float64) / (K - 1)
    table = np.stack([np.interp(u, pos, val[:, c]) for c in range(4)], axis=1)
    return np.clip(table, 0.0, 1.0).astype(np.float32)


def random_tf(K: int, seed: int, alpha_max: float = 1.0, n_points: int = 5,
              air_cut: float = 0.08, min_gap: float = 0.02) -> np.ndarray:
    """Random piecewise-linear RGBA table with ``n_points`` control points at
    U(air_cut, 1) (sorted, consecutive gaps >= ``min_gap`` of the range,
    including the gap to the air cut), RGB ~ U(0,1), alpha ~ U(0, alpha_max).
    Pinned points: value 0 -> (0,0,0,0) and the air cut -> alpha 0 with the
    colour of the first random point."""
    rng = np.random.default_rng(seed)
    while True:
        p = np.sort(rng.uniform(air_cut, 1.0, size=n_points))
        gaps = np.diff(np.concatenate([[air_cut], p]))
        if gaps.min() >= min_gap:
            break
    rgb = rng.uniform(0.0, 1.0, size=(n_points, 3))
    alpha = rng.uniform(0.0, alpha_max, size=n_points)
    positions = [0.0, air_cut] + list(p)
    pts = [[0.0, 0.0, 0.0, 0.0], [rgb[0, 0], rgb[0, 1], rgb[0, 2], 0.0]]
    pts += [[rgb[i, 0], rgb[i, 1], rgb[i, 2], alpha[i]] for i in range(n_points)]
    return tf_from_points(K, positions, pts)


# --------------------------------------------------------------------------
# cameras
# --------------------------------------------------------------------------
def ortho_camera_small(dims=(64, 64, 32), spacing=(1.0, 1.0, 2.0)) -> Camera:
    """Orthographic view along -z from 100 mm above the box centre, up +y,
    half-height 33 mm."""
    c = box_center(dims, spacing)
    return Camera(tuple(c + np.array([0.0, 0.0, 100.0])), tuple(c), (0.0, 1.0, 0.0),
                  False, 0.0, 33.0)


def _orbit_eye(c, dist, az_deg, el_deg):
    az, el = math.radians(az_deg), math.radians(el_deg)
    return c + dist * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])


def orbit_cameras(dims, spacing, n_views: int = 36, elevation_deg: float = 15.0,
                  az_step_deg: float = None, dist_factor: float = 3.0) -> List[Camera]:
    """Orbit about +z (superior axis): azimuth ``az_step*i`` (default 360/n),
    fixed elevation, distance ``dist_factor*R`` with R the bounding-sphere
    radius, fovy = 2*asin(R/D) so the sphere just fits, up = +z."""
    c = box_center(dims, spacing)
    R = bounding_radius(dims, spacing)
    D = dist_factor * R
    fovy = math.degrees(2.0 * math.asin(R / D))
    step = 360.0 / n_views if az_step_deg is None else az_step_deg
    return [Camera(tuple(_orbit_eye(c, D, step * i, elevation_deg)), tuple(c), (0.0, 0.0, 1.0),
                   True, fovy, 0.0) for i in range(n_views)]


def random_camera(rng, dims, spacing) -> Camera:
    """Azimuth U[0,360), elevation U[-60,60], D ~ U[2.5R, 4R], fovy fits the
    bounding sphere, up +z."""
    c = box_center(dims, spacing)
    R = bounding_radius(dims, spacing)
    az = rng.uniform(0.0, 360.0)
    el = rng.uniform(-60.0, 60.0)
    D = rng.uniform(2.5 * R, 4.0 * R)
    fovy = math.degrees(2.0 * math.asin(R / D))
    return Camera(tuple(_orbit_eye(c, D, az, el)), tuple(c), (0.0, 0.0, 1.0), True, fovy, 0.0)


def random_views(seed: int, n_volumes: int = 32, views_per_volume: int = 4,
                 sizes=BATCH_SIZES, spacing=(0.9, 0.9, 1.2)):
    """The uneven batch: volume i has seed 100+i and dims drawn uniformly from
    ``sizes``; each gets ``views_per_volume`` random cameras with a square
    image side drawn from the multiples of 64 in [256, 1024]."""
    rng = np.random.default_rng(seed)
    vols = []
    for i in range(n_volumes):
        dims = tuple(sizes[int(rng.integers(len(sizes)))])
        vols.append(VolumeSpec(dims, tuple(spacing), "u16", 100 + i))
    views = []
    for vi, v in enumerate(vols):
        for _ in range(views_per_volume):
            side = int(64 * rng.integers(4, 17))
            views.append((vi, random_camera(rng, v.dims, v.spacing), side))
    return vols, views


def poisson_requests(seed: int, n: int, rate_hz: float, n_volumes: int, volume_dims: Sequence,
                     spacing=(0.9, 0.9, 1.2)):
    """Poisson arrival stream: exponential gaps with mean 1/rate; each request
    picks a resident volume uniformly, a random camera, a square side from the
    multiples of 64 in [256, 1024] and its own TF seed."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, size=n))
    reqs = []
    for k in range(n):
        vi = int(rng.integers(n_volumes))
        cam = random_camera(rng, volume_dims[vi], spacing)
        side = int(64 * rng.integers(4, 17))
        reqs.append(dict(t=float(t[k]), volume=vi, camera=cam, side=side,
                         tf_seed=int(rng.integers(1 << 30))))
    return reqs
