"""Pins of the oracle's projection ray functions (maximum intensity, X-ray
and average intensity projection; arXiv:1211.5595 Section 2.4 and the ray
function list of Section 4.1) against facts that do not come from the oracle:
hand-derived sample lattices, closed forms on constant and affine fields,
brute force on an impulse, and linearity.

The projected scalar is read back through a ramp table with opacity 1: over a
black background the red channel is (s - vmin) / (vmax - vmin).
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from workloads import Camera

from conftest import GOLDEN

PROJ = ("MIP", "XRAY", "AVERAGE")


def ramp_tf():
    t = np.zeros((2, 4), dtype=np.float32)
    t[:, 3] = 1.0
    t[1, 0] = 1.0
    return t


def decode(img, vmin, vmax):
    return vmin + img[..., 0] * (vmax - vmin)


def slab_chord(o, d, hi):
    """Entry and exit parameters of the ray o + t d (t >= 0) through the box
    [0, hi], by the slab method; None when it misses."""
    t0, t1 = 0.0, math.inf
    for a in range(3):
        if d[a] == 0.0:
            if o[a] < 0.0 or o[a] > hi[a]:
                return None
            continue
        ta, tb = (0.0 - o[a]) / d[a], (hi[a] - o[a]) / d[a]
        t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
    return (t0, t1) if t0 <= t1 else None


def lattice_points(tn, tf, dt):
    """Rule M by hand: midpoints of the full dt-segments and of the remainder."""
    L = tf - tn
    m = int(math.floor(L / dt))
    r = L - m * dt
    s = [tn + (k + 0.5) * dt for k in range(m)]
    w = [1.0] * m
    if r > 0:
        s.append(tn + m * dt + 0.5 * r)
        w.append(r / dt)
    return np.array(s), np.array(w), r / dt


# ---------------------------------------------------------------------------
# the hand-derived 4^3 lattice with f = z
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("rf", PROJ)
def test_projections_on_hand_lattice(orc, rf):
    g = json.load(open(os.path.join(GOLDEN, "lattice_4cube.json")))
    c = g["camera"]
    cam = Camera(tuple(c["eye"]), tuple(c["center"]), tuple(c["up"]), c["perspective"], 0.0,
                 c["ortho_half_height"])
    z = np.arange(4, dtype=np.float64)[:, None, None] * np.ones((4, 4, 4))    # node value = its z (mm)
    vol = orc.Volume(z, g["spacing"])
    vmin, vmax = -1.0, 10.0
    tf = orc.TF(ramp_tf(), vmin, vmax)
    for case in g["cases"]:
        zs, w = np.array(case["z"]), np.array(case["weight"], dtype=np.float64)
        dt = case["step_vox"] * 1.0
        want = {"MIP": zs.max(), "XRAY": dt * (w * zs).sum(), "AVERAGE": (w * zs).sum() / w.sum()}[rf]
        r = orc.render(vol, tf, cam, 3, 3, case["step_vox"], 1.0, ray_function=getattr(orc, rf))
        assert (r.counts == case["count"]).all()
        np.testing.assert_allclose(decode(r.image, vmin, vmax), want, rtol=0, atol=1e-12)
        np.testing.assert_allclose(r.image[..., 3], 1.0, atol=0)


# ---------------------------------------------------------------------------
# closed forms on constant and affine fields, random perspective views
# ---------------------------------------------------------------------------
def _views(seed, dims, sp, n):
    rng = np.random.default_rng(seed)
    return [W.random_camera(rng, dims, sp) for _ in range(n)]


def test_constant_field_closed_forms(orc):
    dims, sp, c = (9, 7, 5), (1.0, 1.5, 2.0), 700.0
    vol = orc.Volume(np.full(dims[::-1], c), sp)
    hi = np.array([(n - 1) * s for n, s in zip(dims, sp)])
    Wd, Hd, step = 16, 12, 0.45
    for cam in _views(3, dims, sp, 3):
        mip = orc.render(vol, orc.TF(ramp_tf(), 0, 1000), cam, Wd, Hd, step, 1.0, ray_function=orc.MIP)
        avg = orc.render(vol, orc.TF(ramp_tf(), 0, 1000), cam, Wd, Hd, step, 1.0, ray_function=orc.AVERAGE)
        xr = orc.render(vol, orc.TF(ramp_tf(), 0, 1e5), cam, Wd, Hd, step, 1.0, ray_function=orc.XRAY)
        n_hit = 0
        for j in range(Hd):
            for i in range(Wd):
                o, d = orc.pixel_ray(cam, Wd, Hd, i, j)
                ch = slab_chord(o, d, hi)
                if ch is None or ch[1] - ch[0] < 1e-9:
                    assert mip.counts[j, i] == 0 or ch is not None
                    continue
                n_hit += 1
                L = ch[1] - ch[0]
                assert decode(mip.image[j, i], 0, 1000) == pytest.approx(c, abs=1e-9)
                assert decode(avg.image[j, i], 0, 1000) == pytest.approx(c, abs=1e-9)
                assert decode(xr.image[j, i], 0, 1e5) == pytest.approx(c * L, rel=1e-10)
        assert n_hit > Wd * Hd // 4


def test_affine_field_closed_forms(orc):
    """f = 3 + 2 qx + 5 qy - 4 qz in index space: trilinear reproduces it, the
    midpoint rule integrates it exactly (X-ray = L f(chord midpoint), average
    = f(chord midpoint)), and its maximum over the lattice sits at the first
    or the last sample."""
    dims, sp = (9, 7, 5), (1.0, 1.5, 2.0)
    k, j, i = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in dims[::-1]], indexing="ij")
    field = 3 + 2 * i + 5 * j - 4 * k
    vol = orc.Volume(field, sp)
    spa = np.array(sp)
    hi = np.array([(n - 1) * s for n, s in zip(dims, sp)])
    f = lambda p: 3 + 2 * p[0] / sp[0] + 5 * p[1] / sp[1] - 4 * p[2] / sp[2]
    vmin, vmax = -100.0, 100.0
    Wd, Hd, step = 16, 12, 0.45
    dt = step * min(sp)
    for cam in _views(5, dims, sp, 3):
        res = {rf: orc.render(vol, orc.TF(ramp_tf(), vmin, vmax if rf != "XRAY" else 2000.0), cam, Wd, Hd, step,
                              1.0, ray_function=getattr(orc, rf)) for rf in PROJ}
        checked = 0
        for jj in range(Hd):
            for ii in range(Wd):
                o, d = orc.pixel_ray(cam, Wd, Hd, ii, jj)
                ch = slab_chord(o, d, hi)
                if ch is None or ch[1] - ch[0] < 1e-6:
                    continue
                s, w, frac = lattice_points(ch[0], ch[1], dt)
                if frac < 1e-6 or frac > 1 - 1e-6:
                    continue                                   # lattice decided by rounding
                mid = o + 0.5 * (ch[0] + ch[1]) * d
                L = ch[1] - ch[0]
                fmax = max(f(o + s[0] * d), f(o + s[-1] * d))
                assert decode(res["MIP"].image[jj, ii], vmin, vmax) == pytest.approx(fmax, abs=1e-9)
                assert decode(res["AVERAGE"].image[jj, ii], vmin, vmax) == pytest.approx(f(mid), abs=1e-9)
                assert decode(res["XRAY"].image[jj, ii], vmin, 2000.0) == pytest.approx(L * f(mid), abs=1e-8)
                assert res["MIP"].counts[jj, ii] == len(s)
                checked += 1
        assert checked > Wd * Hd // 4
    _ = spa


def test_mip_impulse_brute_force(orc):
    """One bright node; an axis-parallel ray through it sees the trilinear
    tent, so the projection is the tent's largest value at the samples."""
    dims, sp = (9, 7, 5), (1.0, 1.0, 1.0)
    v = np.zeros(dims[::-1])
    v[2, 3, 4] = 1000.0                                  # node (x=4, y=3, z=2)
    vol = orc.Volume(v, sp)
    cam = Camera((-5.0, 3.0, 2.0), (0.0, 3.0, 2.0), (0.0, 0.0, 1.0), False, 0.0, 1.0)
    for step in (0.3, 0.45, 0.7):
        r = orc.render(vol, orc.TF(ramp_tf(), 0, 1000), cam, 1, 1, step, 1.0, ray_function=orc.MIP)
        s, w, _ = lattice_points(5.0, 13.0, step)        # ray enters x=0 at t=5, leaves x=8 at t=13
        x = s - 5.0
        want = (1000.0 * np.maximum(0.0, 1.0 - np.abs(x - 4.0))).max()
        assert decode(r.image[0, 0], 0, 1000) == pytest.approx(want, abs=1e-9)


@pytest.mark.parametrize("rf", ("XRAY", "AVERAGE"))
def test_sum_projections_are_linear_in_the_field(orc, rf):
    dims, sp = (11, 8, 6), (0.9, 0.9, 1.2)
    rng = np.random.default_rng(11)
    f = rng.uniform(0, 50, size=dims[::-1])
    g = rng.uniform(0, 50, size=dims[::-1])
    cam = _views(7, dims, sp, 1)[0]
    top = 2000.0 if rf == "XRAY" else 200.0
    out = {}
    for name, field in (("f", f), ("g", g), ("fg", f + 2.5 * g)):
        r = orc.render(orc.Volume(field, sp), orc.TF(ramp_tf(), 0, top), cam, 20, 15, 0.5, 1.0,
                       ray_function=getattr(orc, rf))
        out[name] = decode(r.image, 0, top)
    hit = out["f"] > 0
    assert hit.sum() > 50
    np.testing.assert_allclose(out["fg"][hit], out["f"][hit] + 2.5 * out["g"][hit], rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("rf", PROJ)
def test_projection_miss_gives_background_and_tf_over_background(orc, rf):
    dims, sp = (6, 6, 6), (1.0, 1.0, 1.0)
    vol = orc.Volume(np.full(dims, 10.0), sp)
    t = np.array([[0.2, 0.4, 0.6, 0.25], [0.2, 0.4, 0.6, 0.25]], dtype=np.float32)
    bg = (0.1, 0.2, 0.3, 0.5)
    cam = Camera((2.5, 2.5, -10.0), (2.5, 2.5, 0.0), (0.0, 1.0, 0.0), False, 0.0, 6.0)   # window wider than the box
    r = orc.render(vol, orc.TF(t, 0, 100), cam, 8, 8, 0.5, 1.0, bg=bg, ray_function=getattr(orc, rf))
    hit = r.counts > 0
    assert hit.any() and (~hit).any()
    np.testing.assert_array_equal(r.image[~hit], np.broadcast_to(bg, r.image[~hit].shape))
    a = np.float64(np.float32(0.25))
    want = [a * np.float64(np.float32(c)) + (1 - a) * b for c, b in zip((0.2, 0.4, 0.6), bg[:3])] + \
           [a + (1 - a) * bg[3]]
    np.testing.assert_allclose(r.image[hit], np.broadcast_to(want, r.image[hit].shape), atol=1e-15)


def test_mip_mirror_symmetric_phantom(orc):
    v = W.phantom_small_symmetric(4)
    vol = orc.Volume(v, (1, 1, 2))
    dims = v.shape[::-1]
    c = W.box_center(dims, (1, 1, 2))
    cam = Camera((c[0], c[1] - 300.0, c[2]), tuple(c), (0.0, 0.0, 1.0), True, 20.0, 0.0)
    r = orc.render(vol, orc.TF(W.random_tf(256, 3), 0, 255), cam, 32, 24, 0.5, 1.0, ray_function=orc.MIP)
    np.testing.assert_allclose(r.image, r.image[:, ::-1], atol=1e-12)
