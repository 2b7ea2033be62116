"""Pins of the oracle's thresholding and iso-surface ray functions (the last
two entries of the ray-function list, arXiv:1211.5595 Section 4.1) against
facts that do not come from the oracle: sample lattices and slab geometry
worked out by hand, closed forms on affine fields, and reductions to plain
compositing.
"""
import math

import numpy as np
import pytest

import workloads as W
from workloads import Camera


def const_tf(rgb, a, K=2):
    t = np.zeros((K, 4), dtype=np.float32)
    t[:, :3] = np.asarray(rgb, dtype=np.float32)
    t[:, 3] = np.float32(a)
    return t


def lattice(L, dt):
    m = int(math.floor(L / dt))
    r = L - m * dt
    s = [(k + 0.5) * dt for k in range(m)]
    if r > 0:
        s.append(m * dt + 0.5 * r)
    return np.array(s), m, r


# ---------------------------------------------------------------------------
# thresholding
# ---------------------------------------------------------------------------
def test_threshold_wide_window_equals_compositing(orc):
    v = W.phantom_small(3)
    vol = orc.Volume(v, (1, 1, 2))
    tf = orc.TF(W.random_tf(256, 5), 0, 255)
    cam = W.ortho_camera_small()
    a = orc.render(vol, tf, cam, 48, 40, 0.5, 0.99)
    b = orc.render(vol, tf, cam, 48, 40, 0.5, 0.99, ray_function=orc.THRESHOLD, iso_value=-1.0, iso_high=300.0)
    assert np.array_equal(a.image, b.image) and np.array_equal(a.counts, b.counts)


def test_threshold_empty_window_gives_background(orc):
    v = W.phantom_small(3)
    vol = orc.Volume(v, (1, 1, 2))
    tf = orc.TF(W.random_tf(256, 5), 0, 255)
    bg = (0.1, 0.2, 0.3, 0.4)
    r = orc.render(vol, tf, W.ortho_camera_small(), 32, 32, 0.5, 0.99, bg=bg, ray_function=orc.THRESHOLD,
                   iso_value=300.0, iso_high=400.0)
    np.testing.assert_array_equal(r.image, np.broadcast_to(bg, r.image.shape))


@pytest.mark.parametrize("lo,hi", [(150.0, 250.0), (50.0, 150.0), (120.0, 180.0), (100.0, 100.0)])
def test_threshold_two_material_slab_by_hand(orc, lo, hi):
    """Nodes x < 4 hold 100, x >= 4 hold 200 (index space); an orthographic
    ray along +x samples the piecewise-linear profile 100 -> 200 across the
    cell [3, 4].  With a constant table (colour c, opacity a) the result is
    c (1 - (1-a)^n) over the background, n = number of samples whose value is
    in the window -- counted here from the hand lattice."""
    nx, sp = 10, 1.0
    v = np.zeros((3, 3, nx))
    v[:, :, :4] = 100.0
    v[:, :, 4:] = 200.0
    vol = orc.Volume(v, (sp, 1.0, 1.0))
    c, a = (0.7, 0.5, 0.3), 0.125
    tf = orc.TF(const_tf(c, a), 0, 255)
    cam = Camera((-5.0, 1.0, 1.0), (0.0, 1.0, 1.0), (0.0, 0.0, 1.0), False, 0.0, 0.5)
    step = 0.35
    s, m, r = lattice((nx - 1) * sp, step)
    x = s                                    # ray enters x = 0 at t = 5
    val = np.where(x <= 3, 100.0, np.where(x >= 4, 200.0, 100.0 + 100.0 * (x - 3)))
    inside = (val >= lo) & (val <= hi)
    w = np.ones(len(s))
    if r > 0:
        w[-1] = r / step
    got = orc.render(vol, tf, cam, 1, 1, step, 1.0, ray_function=orc.THRESHOLD, iso_value=lo, iso_high=hi)
    a32 = float(np.float32(a))
    Tw = np.prod([(1 - a32) ** wi if ins else 1.0 for ins, wi in zip(inside, w)])
    np.testing.assert_allclose(got.image[0, 0, :3], np.float32(c).astype(np.float64) * (1 - Tw), atol=1e-12)
    np.testing.assert_allclose(got.image[0, 0, 3], 1 - Tw, atol=1e-12)
    assert got.counts[0, 0] == len(s)


def test_threshold_tie_flag_on_a_window_edge(orc):
    """A sample whose value sits on the window edge is decided by rounding:
    the oracle must flag the pixel (tie bit 3)."""
    v = np.zeros((3, 3, 6))
    v[:, :, :] = np.arange(6)[None, None, :] * 10.0      # f = 10 x
    vol = orc.Volume(v, (1.0, 1.0, 1.0))
    cam = Camera((-5.0, 1.0, 1.0), (0.0, 1.0, 1.0), (0.0, 0.0, 1.0), False, 0.0, 0.5)
    tf = orc.TF(const_tf((1, 1, 1), 0.1), 0, 100)
    # step 0.5: samples at x = 0.25, 0.75, ... -> values 2.5, 7.5, 12.5, ...
    hit = orc.render(vol, tf, cam, 1, 1, 0.5, 1.0, ray_function=orc.THRESHOLD, iso_value=12.5, iso_high=30.0)
    off = orc.render(vol, tf, cam, 1, 1, 0.5, 1.0, ray_function=orc.THRESHOLD, iso_value=11.0, iso_high=30.0)
    assert hit.tie[0, 0] & 8 and not (off.tie[0, 0] & 8)


# ---------------------------------------------------------------------------
# iso-surface
# ---------------------------------------------------------------------------
def slab_chord(o, d, hi):
    t0, t1 = 0.0, math.inf
    for ax in range(3):
        if d[ax] == 0.0:
            if o[ax] < 0.0 or o[ax] > hi[ax]:
                return None
            continue
        ta, tb = (0.0 - o[ax]) / d[ax], (hi[ax] - o[ax]) / d[ax]
        t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
    return (t0, t1) if t0 <= t1 else None


@pytest.mark.parametrize("seed", range(4))
def test_iso_affine_field_closed_form(orc, seed):
    """f = b + g.q (index space) is reproduced exactly by trilinear
    interpolation and by the linear refinement, so the surface is hit where
    the ray first reaches the iso-value after a lattice sample does, and the
    central-difference normal is the exact gradient: the shade is
    c (0.2 + 0.8 |g_mm . d| / |g_mm|), g_mm = g / spacing."""
    rng = np.random.default_rng(40 + seed)
    dims, sp = (17, 15, 13), np.array([1.0, 1.5, 2.0])
    cam = W.random_camera(rng, dims, tuple(sp))
    g = rng.uniform(-20, 20, 3)
    if g @ ((np.array(cam.eye) - np.array(cam.center)) / sp) > 0:
        g = -g                                   # values rise away from the eye: rays cross inside
    b = 100.0
    k, j, i = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in dims[::-1]], indexing="ij")
    field = b + g[0] * i + g[1] * j + g[2] * k
    vol = orc.Volume(field, tuple(sp))
    lo_f = b + float(np.minimum(g, 0) @ (np.array(dims) - 1))
    iso = lo_f + 0.55 * float(np.abs(g) @ (np.array(dims) - 1))       # a plane through the middle
    c = (0.9, 0.6, 0.3)
    tf = orc.TF(const_tf(c, 0.5), -2000, 2000)
    hi = (np.array(dims) - 1) * sp
    Wd, Hd, step = 48, 40, 0.4
    dt = step * sp.min()
    r = orc.render(orc.Volume(field, tuple(sp)), tf, cam, Wd, Hd, step, 1.0, ray_function=orc.ISO, iso_value=iso)
    gmm = g / sp
    checked = 0
    for jj in range(Hd):
        for ii in range(Wd):
            o, d = orc.pixel_ray(cam, Wd, Hd, ii, jj)
            ch = slab_chord(o, d, hi)
            if ch is None or ch[1] - ch[0] < 1e-6 or r.tie[jj, ii]:
                continue
            s, m, rem = lattice(ch[1] - ch[0], dt)
            vals = b + ((o[None, :] + (ch[0] + s)[:, None] * d[None, :]) / sp[None, :]) @ g
            first = np.nonzero(vals >= iso)[0]
            if len(first) == 0:
                np.testing.assert_array_equal(r.image[jj, ii], 0.0)
                assert r.counts[jj, ii] == len(s)
                continue
            assert r.counts[jj, ii] == first[0] + 1
            k0 = first[0]
            t_hit = s[0] if k0 == 0 else s[k0 - 1] + (iso - vals[k0 - 1]) / (vals[k0] - vals[k0 - 1]) * (s[k0] - s[k0 - 1])
            q_hit = (o + (ch[0] + t_hit) * d) / sp
            if (q_hit - 0.5 < 0).any() or (q_hit + 0.5 > np.array(dims) - 1).any():
                continue                  # the central differences reach past a face and are clamped
            shade = 0.2 + 0.8 * abs(gmm @ d) / np.linalg.norm(gmm)
            want = np.float32(c).astype(np.float64) * shade
            np.testing.assert_allclose(r.image[jj, ii, :3], want, atol=1e-12)
            assert r.image[jj, ii, 3] == 1.0
            checked += 1
    assert checked > 10


def test_iso_hit_point_refined_on_the_ray(orc):
    """Along +x through f = 10 x the refined hit of iso = 33 is x = 3.3 exactly:
    the normal is -x, |n.d| = 1, so the shade is the full colour; a field
    that never reaches the iso-value shows the background."""
    v = np.zeros((3, 3, 8))
    v[:, :, :] = np.arange(8)[None, None, :] * 10.0
    vol = orc.Volume(v, (1.0, 1.0, 1.0))
    cam = Camera((-5.0, 1.0, 1.0), (0.0, 1.0, 1.0), (0.0, 0.0, 1.0), False, 0.0, 0.5)
    tf = orc.TF(const_tf((0.25, 0.5, 0.75), 1.0), 0, 100)
    r = orc.render(vol, tf, cam, 1, 1, 0.5, 1.0, ray_function=orc.ISO, iso_value=33.0)
    np.testing.assert_allclose(r.image[0, 0], [0.25, 0.5, 0.75, 1.0], atol=1e-12)
    assert r.counts[0, 0] == 8                         # samples at 0.25 ... 3.25 (< 33), then 3.75
    bg = (0.1, 0.1, 0.1, 0.1)
    miss = orc.render(vol, tf, cam, 1, 1, 0.5, 1.0, bg=bg, ray_function=orc.ISO, iso_value=80.0)
    np.testing.assert_array_equal(miss.image[0, 0], bg)
    assert miss.counts[0, 0] == 14


def test_iso_hit_at_the_first_sample_is_not_refined(orc):
    """When the first sample already reaches the iso-value the ray starts
    inside the surface: the hit is that sample (no previous one to refine
    from), shaded by the exact gradient there."""
    v = np.zeros((3, 3, 8))
    v[:, :, :] = 50.0 + np.arange(8)[None, None, :] * 10.0     # f = 50 + 10 x
    vol = orc.Volume(v, (1.0, 1.0, 1.0))
    d = np.array([0.6, 0.0, 0.8])
    o = np.array([4.0, 1.0, 1.0]) - 5.0 * d                        # enters through z = 0 at x = 3.25
    cam = Camera(tuple(o), tuple(o + d), (0.0, 1.0, 0.0), False, 0.0, 0.25)
    tf = orc.TF(const_tf((1.0, 1.0, 1.0), 1.0), 0, 100)
    r = orc.render(vol, tf, cam, 1, 1, 0.5, 1.0, ray_function=orc.ISO, iso_value=40.0)
    np.testing.assert_allclose(r.image[0, 0, :3], 0.2 + 0.8 * 0.6, atol=1e-12)
    assert r.counts[0, 0] == 1


def test_iso_band_covers_the_rounding_of_the_normal(orc):
    """On a noisy field the band is never empty around the value and widens
    where the gradient is weak."""
    rng = np.random.default_rng(9)
    v = rng.normal(1000.0, 20.0, size=(20, 24, 28))
    vol = orc.Volume(v, (1.0, 1.0, 1.0))
    tf = orc.TF(W.random_tf(256, 7), 900, 1100)
    cam = W.random_camera(rng, (28, 24, 20), (1.0, 1.0, 1.0))
    r = orc.render(vol, tf, cam, 30, 30, 0.5, 1.0, ray_function=orc.ISO, iso_value=1010.0, want_band=True)
    assert (r.band_lo <= r.image).all() and (r.image <= r.band_hi).all()
    assert (r.band_hi - r.band_lo).max() > 0.0
