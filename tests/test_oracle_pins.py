"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test checks one part of the method (arXiv:1211.5595, Sections 3.2, 4.1,
4.2) against a hand derivation, a closed form, an invariant or a library
routine, chosen so that a plausible slip (a dropped term, a wrong sign or
index, a transposed operand, a shifted sample) fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import ndimage

import workloads as W
from workloads import Camera

from conftest import GOLDEN


def const_tf(K, rgb, a):
    t = np.zeros((K, 4), dtype=np.float32)
    t[:, :3] = np.asarray(rgb, dtype=np.float32)
    t[:, 3] = np.float32(a)
    return t


# ---------------------------------------------------------------------------
# step 1: ray generation (Section 4.1, Section 6 camera settings)
# ---------------------------------------------------------------------------
def test_pixel_rays_hand_values(orc):
    g = json.load(open(os.path.join(GOLDEN, "rays_hand.json")))
    for c in g["perspective"]:
        cam = Camera((0, 0, 0), (0, 0, -1), (0, 1, 0), True, 90.0)
        o, d = orc.pixel_ray(cam, c["W"], c["H"], c["i"], c["j"])
        x, y = c["plane_xy"]
        want = np.array([x, y, -1.0]) / math.sqrt(x * x + y * y + 1.0)
        np.testing.assert_allclose(o, 0.0, atol=0)
        np.testing.assert_allclose(d, want, rtol=0, atol=1e-15)
    for c in g["orthographic"]:
        cam = Camera((0, 0, 5), (0, 0, 0), (0, 1, 0), False, 0.0, 3.0)
        o, d = orc.pixel_ray(cam, c["W"], c["H"], c["i"], c["j"])
        x, y = c["origin_xy"]
        np.testing.assert_allclose(o, [x, y, 5.0], atol=1e-15)
        np.testing.assert_allclose(d, [0, 0, -1], atol=0)


def test_pixel_rays_mirror_and_unit(orc):
    rng = np.random.default_rng(5)
    for _ in range(20):
        eye = rng.normal(size=3) * 50
        cam = Camera(tuple(eye), (0, 0, 0), (0, 0, 1), True, float(rng.uniform(10, 120)))
        w, u, v = orc.camera_frame(cam)
        Wd, Hd = int(rng.integers(1, 40)), int(rng.integers(1, 40))
        i, j = int(rng.integers(Wd)), int(rng.integers(Hd))
        _, d1 = orc.pixel_ray(cam, Wd, Hd, i, j)
        _, d2 = orc.pixel_ray(cam, Wd, Hd, Wd - 1 - i, j)
        assert abs(np.linalg.norm(d1) - 1) < 1e-15
        # mirrored columns: same w and v components, opposite u component
        assert abs(d1 @ w - d2 @ w) < 1e-14 and abs(d1 @ v - d2 @ v) < 1e-14
        assert abs(d1 @ u + d2 @ u) < 1e-14
        # right-handed orthonormal frame with v in the plane of w and up
        np.testing.assert_allclose(np.cross(u, v), -w, atol=1e-15)
        assert np.cross(w, (0, 0, 1)) @ v == pytest.approx(0, abs=1e-14)


def test_camera_invalid(orc):
    with pytest.raises(ValueError):
        orc.camera_frame(Camera((1, 2, 3), (1, 2, 3), (0, 0, 1), True, 30))
    with pytest.raises(ValueError):
        orc.camera_frame(Camera((0, 0, 5), (0, 0, 0), (0, 0, 1), True, 30))


# ---------------------------------------------------------------------------
# step 1: ray / volume intersection, brute force
# ---------------------------------------------------------------------------
def _inside(p, hi, eps=1e-9):
    return np.all(p >= -eps, axis=-1) & np.all(p <= hi + eps, axis=-1)


def test_box_clip_brute_force(orc):
    rng = np.random.default_rng(7)
    hi = np.array([3.0, 5.0, 2.0])
    n_hit = 0
    for trial in range(200):
        o = rng.uniform(-6, 9, size=3)
        d = rng.uniform(-1, [4, 6, 3]) - o if trial % 4 else rng.normal(size=3)
        d /= np.linalg.norm(d)
        hit, tn, tf = orc.box_clip(o, d, hi)
        ts = np.linspace(0, 30, 150001)
        inside = _inside(o[None, :] + ts[:, None] * d[None, :], hi)
        step = ts[1] - ts[0]
        if not inside.any():
            assert not hit or tf - tn < 2 * step
            continue
        n_hit += 1
        assert hit
        assert abs(tn - ts[np.argmax(inside)]) <= step
        assert abs(tf - ts[len(ts) - 1 - np.argmax(inside[::-1])]) <= step
    assert n_hit > 50


def test_box_clip_special_cases(orc):
    hi = np.array([3.0, 3.0, 3.0])
    # direction component exactly zero, inside that slab: chord along z
    hit, tn, tf = orc.box_clip([1.0, 2.0, -4.0], [0.0, 0.0, 1.0], hi)
    assert hit and tn == 4.0 and tf == 7.0
    # zero component, outside the slab: miss
    hit, _, _ = orc.box_clip([4.0, 2.0, -4.0], [0.0, 0.0, 1.0], hi)
    assert not hit
    # eye inside: sampling starts at the eye
    hit, tn, tf = orc.box_clip([1.0, 1.0, 1.0], [0.0, 0.0, 1.0], hi)
    assert hit and tn == 0.0 and tf == 2.0
    # box behind the eye: miss
    hit, _, _ = orc.box_clip([1.0, 1.0, 5.0], [0.0, 0.0, 1.0], hi)
    assert not hit


# ---------------------------------------------------------------------------
# step 1: evenly spaced samples, hand counts on a 4^3 volume
# ---------------------------------------------------------------------------
def test_lattice_hand_counts_4cube(orc):
    g = json.load(open(os.path.join(GOLDEN, "lattice_4cube.json")))
    c = g["camera"]
    cam = Camera(tuple(c["eye"]), tuple(c["center"]), tuple(c["up"]), c["perspective"], 0.0,
                 c["ortho_half_height"])
    vol = orc.Volume(np.zeros((4, 4, 4)), g["spacing"])
    tf = orc.TF(const_tf(2, (1, 1, 1), 0.0), 0, 1)
    for case in g["cases"]:
        r = orc.render(vol, tf, cam, 3, 3, case["step_vox"], 1.0)
        assert (r.counts == case["count"]).all()
        for j in range(3):
            for i in range(3):
                rec = orc.trace_ray(vol, tf, cam, 3, 3, i, j, case["step_vox"], 1.0)
                assert len(rec) == case["count"]
                np.testing.assert_allclose(rec[:, 4], case["z"], atol=1e-12)        # q_z
                np.testing.assert_allclose(rec[:, 1], case["weight"], atol=1e-12)   # weight
                np.testing.assert_allclose(rec[:, 2], g["pixel_x_mm"][j][i], atol=1e-12)
                np.testing.assert_allclose(rec[:, 3], g["pixel_y_mm"][j][i], atol=1e-12)


def test_lattice_remainder(orc):
    for L, dt, n, m, r in [(3.0, 0.5, 6, 6, 0.0), (3.0, 0.4, 8, 7, 0.2), (0.1, 0.5, 1, 0, 0.1),
                           (1.0, 1.0, 1, 1, 0.0)]:
        nn, mm, rr = orc.lattice(L, dt)
        assert (nn, mm) == (n, m) and abs(rr - r) < 1e-12


def test_samples_evenly_spaced_in_mm(orc):
    """Perspective ray through an anisotropic volume: consecutive samples are
    dt = step*min(spacing) apart in millimetres, the first sits dt/2 past the
    box entry found by brute force, and all lie in the box."""
    dims, sp = (20, 16, 12), (0.9, 1.1, 1.7)
    vol = orc.Volume(np.zeros(dims[::-1]), sp)
    tf = orc.TF(const_tf(2, (1, 1, 1), 0.0), 0, 1)
    cams = W.orbit_cameras(dims, sp, 5, elevation_deg=25)
    dt = 0.3 * 0.9
    for cam in cams:
        rec = orc.trace_ray(vol, tf, cam, 31, 17, 13, 9, 0.3, 1.0)
        assert len(rec) > 10
        p = rec[:, 2:5] * np.array(sp)
        gaps = np.linalg.norm(np.diff(p[:-1], axis=0), axis=1)
        np.testing.assert_allclose(gaps, dt, atol=1e-12)
        hi = (np.array(dims) - 1) * np.array(sp)
        assert _inside(p, hi, 1e-9).all()
        o, d = orc.pixel_ray(cam, 31, 17, 13, 9)
        ts = np.linspace(0, 2000, 2000001)
        ins = _inside(o + ts[:, None] * d, hi)
        t_entry = ts[np.argmax(ins)]
        assert abs(np.linalg.norm(p[0] - o) - (t_entry + dt / 2)) < 2e-3


# ---------------------------------------------------------------------------
# step 2: trilinear resampling (Section 3.2)
# ---------------------------------------------------------------------------
def test_trilinear_exact_on_affine(orc):
    rng = np.random.default_rng(3)
    nz, ny, nx = 6, 7, 9
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    a, b, c, d0 = 1.25, -2.5, 0.75, 10.0
    vol = orc.Volume(a * i + b * j + c * k + d0, (1, 1, 1))
    for _ in range(200):
        q = rng.uniform([0, 0, 0], [nx - 1, ny - 1, nz - 1])
        assert orc.trilinear(vol, q) == pytest.approx(a * q[0] + b * q[1] + c * q[2] + d0, abs=1e-12)
    # outside the box the position is clamped to the nearest face
    assert orc.trilinear(vol, [-3.0, 2.0, 1.0]) == pytest.approx(b * 2 + c + d0, abs=1e-12)
    assert orc.trilinear(vol, [nx + 4.0, 2.0, 1.0]) == pytest.approx(a * (nx - 1) + b * 2 + c + d0, abs=1e-12)


def test_trilinear_impulse_is_tent(orc):
    f = np.zeros((5, 5, 5))
    f[2, 3, 1] = 1.0   # z=2, y=3, x=1
    vol = orc.Volume(f, (1, 1, 1))
    rng = np.random.default_rng(4)
    for _ in range(200):
        q = rng.uniform(0, 4, size=3)
        want = max(0, 1 - abs(q[0] - 1)) * max(0, 1 - abs(q[1] - 3)) * max(0, 1 - abs(q[2] - 2))
        assert orc.trilinear(vol, q) == pytest.approx(want, abs=1e-14)


def test_trilinear_matches_scipy(orc):
    rng = np.random.default_rng(9)
    f = rng.uniform(0, 4095, size=(7, 11, 13))
    vol = orc.Volume(f, (0.9, 0.9, 1.2))
    q = rng.uniform(-0.5, [12.5, 10.5, 6.5], size=(500, 3))
    want = ndimage.map_coordinates(f, [q[:, 2], q[:, 1], q[:, 0]], order=1, mode="nearest")
    got = np.array([orc.trilinear(vol, x) for x in q])
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-9)


# ---------------------------------------------------------------------------
# step 2: classification (Sections 2.6, 6)
# ---------------------------------------------------------------------------
def test_classify_matches_numpy_interp(orc):
    rng = np.random.default_rng(11)
    for K, vmin, vmax in [(2, 0, 1), (256, 0, 255), (4096, 0, 4095), (37, -5.5, 130.25)]:
        table = rng.uniform(0, 1, size=(K, 4)).astype(np.float32)
        tf = orc.TF(table, vmin, vmax)
        xs = np.linspace(vmin, vmax, K).astype(np.float64)
        for val in np.concatenate([rng.uniform(vmin - 10, vmax + 10, 100), [vmin, vmax]]):
            got = orc.classify(tf, val)
            want = [np.interp(val, xs, table[:, c].astype(np.float64)) for c in range(4)]
            np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


def test_classify_identity_ramp(orc):
    K = 4096
    ramp = np.repeat((np.arange(K) / (K - 1)).astype(np.float32)[:, None], 4, axis=1)
    tf = orc.TF(ramp, 0, 4095)
    for val in [0.0, 1.0, 17.5, 2047.25, 4094.9, 4095.0, 5000.0, -3.0]:
        want = min(max(val / 4095.0, 0.0), 1.0)
        np.testing.assert_allclose(orc.classify(tf, val), want, atol=1e-7)


# ---------------------------------------------------------------------------
# step 3: compositing (Section 4.2)
# ---------------------------------------------------------------------------
SLAB_CAM = Camera((1.5, 1.5, -10.0), (1.5, 1.5, 0.0), (0, 1, 0), False, 0.0, 1.0)


@pytest.mark.parametrize("step,a", [(0.5, 0.1), (0.25, 0.02), (0.4, 0.3), (0.7, 0.05), (0.5, 0.0), (0.5, 1.0)])
def test_constant_slab_closed_form(orc, step, a):
    """Uniform volume, constant TF (c, a), chord L = 3 mm: accumulated opacity
    1-(1-a)^(L/dt) (n = L/dt samples, the last one fractional) and colour c
    times that opacity."""
    vol = orc.Volume(np.full((4, 4, 4), 7.0), (1, 1, 1))
    c = (0.2, 0.5, 0.9)
    tf = orc.TF(const_tf(8, c, a), 0, 10)
    r = orc.render(vol, tf, SLAB_CAM, 2, 2, step, 1.0)
    a = float(np.float32(a))  # the table holds binary32 opacities
    A = 1 - (1 - a) ** (3.0 / step)
    np.testing.assert_allclose(r.image[..., 3], A, atol=1e-12)
    for ch in range(3):
        np.testing.assert_allclose(r.image[..., ch], float(np.float32(c[ch])) * A, atol=1e-12)


def test_constant_slab_over_background(orc):
    """The slab seen over a premultiplied background: the 'over' operator,
    rgb = c*A + (1-A)*bg_rgb and alpha = A + (1-A)*bg_a."""
    vol = orc.Volume(np.full((4, 4, 4), 7.0), (1, 1, 1))
    c, a, bg = (0.2, 0.5, 0.9), 0.1, (0.3, 0.05, 0.6, 0.7)
    r = orc.render(vol, orc.TF(const_tf(8, c, a), 0, 10), SLAB_CAM, 2, 2, 0.5, 1.0, bg=bg)
    A = 1 - (1 - float(np.float32(a))) ** 6
    for ch in range(3):
        np.testing.assert_allclose(r.image[..., ch], float(np.float32(c[ch])) * A + (1 - A) * bg[ch], atol=1e-12)
    np.testing.assert_allclose(r.image[..., 3], A + (1 - A) * bg[3], atol=1e-12)


def test_constant_colour_invariant(orc):
    """Constant TF colour c with varying opacity: rgb = c * alpha (black bg)."""
    v = W.phantom_small(1)
    rng = np.random.default_rng(2)
    table = const_tf(256, (0.3, 0.6, 0.1), 0.0)
    table[:, 3] = rng.uniform(0, 0.2, 256).astype(np.float32)
    r = orc.render(orc.Volume(v, (1, 1, 2)), orc.TF(table, 0, 255), W.ortho_camera_small(), 64, 64, 0.5, 0.99)
    for ch, c in enumerate((0.3, 0.6, 0.1)):
        np.testing.assert_allclose(r.image[..., ch], np.float32(c) * r.image[..., 3], atol=1e-12)


def test_front_to_back_equals_back_to_front(orc):
    """Eq. (4) sums attenuated emissions in the paper's back-to-front order;
    the oracle accumulates front-to-back.  Rebuild eq. (4) from the traced
    per-sample emissions and opacities, from the far end to the eye."""
    v = W.phantom_small(1)
    vol = orc.Volume(v, (1, 1, 2))
    tf = orc.TF(W.random_tf(256, 2), 0, 255)
    cam = W.ortho_camera_small()
    r = orc.render(vol, tf, cam, 32, 32, 0.5, 1.0)
    for (i, j) in [(16, 16), (10, 20), (5, 5), (25, 12)]:
        rec = orc.trace_ray(vol, tf, cam, 32, 32, i, j, 0.5, 1.0)
        I = np.zeros(3)
        Tb = 1.0
        for k in range(len(rec) - 1, -1, -1):
            a = rec[k, 10]
            I = rec[k, 6:9] * a + (1 - a) * I
            Tb *= (1 - a)
        np.testing.assert_allclose(r.image[j, i, :3], I, atol=1e-12)
        assert r.image[j, i, 3] == pytest.approx(1 - Tb, abs=1e-12)


def test_converges_to_emission_absorption_integral(orc):
    """Eq. (5): with alpha = 1-exp(-kappa*dt) and constant emission colour c,
    the pixel tends to c*(1-exp(-integral of kappa)).  kappa(v) = v/100 per mm
    on the field v(z) = z^2 (z in mm) along a chord z in [0, 3]; the integral
    is 9/100 = 0.09.  Midpoint samples converge at O(dt^2)."""
    nz = 301
    z = np.arange(nz) * 0.01
    f = np.broadcast_to((z ** 2)[:, None, None], (nz, 4, 4)).copy()
    vol = orc.Volume(f, (1.0, 1.0, 0.01))
    exact = 1 - math.exp(-0.09)
    errs = []
    for step in (40.0, 20.0, 10.0):  # in units of the finest spacing (0.01 mm)
        dt = step * 0.01
        K = 20001
        vals = np.linspace(0, 9, K)
        table = np.zeros((K, 4), dtype=np.float32)
        table[:, :3] = 1.0
        table[:, 3] = (1 - np.exp(-vals / 100 * dt)).astype(np.float32)
        tf = orc.TF(table, 0, 9)
        cam = Camera((1.5, 1.5, -5.0), (1.5, 1.5, 0.0), (0, 1, 0), False, 0.0, 1.0)
        r = orc.render(vol, tf, cam, 1, 1, step, 1.0)
        errs.append(abs(r.image[0, 0, 3] - exact))
    assert errs[0] < 5e-4
    assert errs[1] < errs[0] / 3 and errs[2] < errs[1] / 3


# ---------------------------------------------------------------------------
# early termination, background, whole-image invariants
# ---------------------------------------------------------------------------
def test_early_termination_bound(orc):
    v = W.phantom_brain(11, dims=(48, 48, 30))
    vol = orc.Volume(v, (0.9, 0.9, 1.2))
    tf = orc.TF(W.random_tf(4096, 12, alpha_max=0.3), 0, 4095)
    cam = W.orbit_cameras((48, 48, 30), (0.9, 0.9, 1.2), 4)[1]
    et = orc.render(vol, tf, cam, 48, 48, 0.5, 0.99)
    full = orc.render(vol, tf, cam, 48, 48, 0.5, 1.0)
    cmax = tf.rgba[:, :3].max()
    assert (np.abs(et.image[..., :3] - full.image[..., :3]) <= 0.01 * cmax + 1e-12).all()
    assert (np.abs(et.image[..., 3] - full.image[..., 3]) <= 0.01 + 1e-12).all()
    assert (et.counts <= full.counts).all() and (et.counts < full.counts).any()


@pytest.mark.parametrize("a,cutoff", [(0.1, 0.99), (0.05, 0.9), (0.3, 0.5)])
def test_early_termination_constant_slab_count(orc, a, cutoff):
    """Opacity after n samples is 1-(1-a)^n, so the ray stops after
    n_ET = ceil(ln(1-cutoff)/ln(1-a)) samples."""
    nz = 401
    vol = orc.Volume(np.full((nz, 4, 4), 1.0), (1, 1, 1))
    tf = orc.TF(const_tf(4, (1, 1, 1), a), 0, 2)
    cam = Camera((1.5, 1.5, -10.0), (1.5, 1.5, 0.0), (0, 1, 0), False, 0.0, 1.0)
    r = orc.render(vol, tf, cam, 1, 1, 0.5, cutoff)
    a = float(np.float32(a))  # the table holds binary32 opacities
    n_et = math.ceil(math.log(1 - cutoff) / math.log(1 - a))
    assert r.counts[0, 0] == n_et
    assert r.image[0, 0, 3] == pytest.approx(1 - (1 - a) ** n_et, abs=1e-12)


def test_tie_band_brackets_stopping_points(orc):
    """a = 0.9, cutoff 0.99: after two samples the opacity is 0.99 up to
    rounding, so stopping after sample 2 or 3 are both acceptable."""
    vol = orc.Volume(np.full((40, 4, 4), 1.0), (1, 1, 1))
    tf = orc.TF(const_tf(4, (1, 1, 1), 0.9), 0, 2)
    cam = Camera((1.5, 1.5, -10.0), (1.5, 1.5, 0.0), (0, 1, 0), False, 0.0, 1.0)
    r = orc.render(vol, tf, cam, 1, 1, 1.0, 0.99, tie_delta=1e-6, want_band=True)
    t = 1 - float(np.float32(0.9))
    a2, a3 = 1 - t ** 2, 1 - t ** 3
    assert r.tie[0, 0] & 1
    assert r.counts[0, 0] == 3          # 1-t^2 falls just short of 0.99 in binary32 opacity
    assert r.band_lo[0, 0, 3] == pytest.approx(a2, abs=1e-15)
    assert r.band_hi[0, 0, 3] == pytest.approx(a3, abs=1e-15)


def _slab_1px(orc, a, cutoff, tie_delta, nz=40):
    vol = orc.Volume(np.full((nz, 4, 4), 1.0), (1, 1, 1))
    tf = orc.TF(const_tf(4, (1, 1, 1), a), 0, 2)
    cam = Camera((1.5, 1.5, -10.0), (1.5, 1.5, 0.0), (0, 1, 0), False, 0.0, 1.0)
    return orc.render(vol, tf, cam, 1, 1, 1.0, cutoff, tie_delta=tie_delta, want_band=True)


@pytest.mark.parametrize("a,cutoff,n_stop", [(0.5, 0.75, 2), (0.5, 0.875, 3), (0.75, 0.9375, 2), (1.0, 1.0, 1),
                                             (1.0, 0.5, 1)])
@pytest.mark.parametrize("tie_delta", [0.0, 1e-6])
def test_cutoff_reached_exactly_stops(orc, a, cutoff, n_stop, tie_delta):
    """The ray stops after the first sample with 1-T >= cutoff, equality
    included.  Opacities that are powers of two make 1-T exact in binary64:
    a = 0.5 gives 1-T = 0.5, 0.75, 0.875, ... and a = 1 gives 1-T = 1 after
    one sample, so a cutoff equal to one of these values must stop the ray on
    that very sample (a strict test would take one sample more -- or, for a
    = 1 at cutoff 1, never stop).  The counted samples and the pixel are those
    of the stopping sample."""
    r = _slab_1px(orc, a, cutoff, tie_delta)
    assert r.counts[0, 0] == n_stop
    assert r.image[0, 0, 3] == 1 - (1 - a) ** n_stop


def test_tie_band_reaches_past_the_stopping_sample(orc):
    """Binary64 stops at sample 2 with 1-T = 0.75 just above the cutoff
    0.75 - 1e-7, inside the band [cutoff - d, cutoff + d) with d = 1e-6: a
    binary32 ray may round its opacity below the cutoff and take sample 3.
    The band must therefore run on past the stopping sample up to the first
    state with 1-T >= cutoff + d, the state after sample 3 (1-T = 0.875),
    while the pixel and count stay those of sample 2."""
    r = _slab_1px(orc, 0.5, 0.75 - 1e-7, 1e-6)
    assert r.counts[0, 0] == 2
    assert r.image[0, 0, 3] == 0.75
    assert r.tie[0, 0] & 1
    assert r.band_lo[0, 0, 3] == 0.75
    assert r.band_hi[0, 0, 3] == 0.875
    assert r.band_hi[0, 0, 0] == 0.875   # white colour: rgb equals the opacity


def test_tie_band_starts_before_the_cutoff(orc):
    """The mirror case: binary64 opacity after sample 2 (0.75) sits just below
    the cutoff 0.75 + 1e-7, so binary64 stops at sample 3, yet a binary32 ray
    may stop at sample 2; the band opens at sample 2 and closes at sample 3."""
    r = _slab_1px(orc, 0.5, 0.75 + 1e-7, 1e-6)
    assert r.counts[0, 0] == 3
    assert r.image[0, 0, 3] == 0.875
    assert r.tie[0, 0] & 1
    assert r.band_lo[0, 0, 3] == 0.75
    assert r.band_hi[0, 0, 3] == 0.875


def test_tie_band_edges_include_equality(orc):
    """The band opens at the first state with 1-T >= cutoff - d and closes at
    the first with 1-T >= cutoff + d, both inclusive.  a = 0.5 gives the exact
    opacities 0.5, 0.75, 0.875, 0.9375; cutoff 0.8125 with d = 0.0625 puts
    both edges exactly on them (0.75 and 0.875)."""
    r = _slab_1px(orc, 0.5, 0.8125, 0.0625)
    assert r.counts[0, 0] == 3
    assert r.band_lo[0, 0, 3] == 0.75
    assert r.band_hi[0, 0, 3] == 0.875


def test_tie_band_closed_when_far_from_cutoff(orc):
    """With the stopping opacity well clear of the cutoff (0.75 against
    0.7, d = 1e-6) there is no tie: the band is the single stopping state."""
    r = _slab_1px(orc, 0.5, 0.7, 1e-6)
    assert r.counts[0, 0] == 2
    assert not (r.tie[0, 0] & 1)
    assert r.band_lo[0, 0, 3] == 0.75 and r.band_hi[0, 0, 3] == 0.75


def test_transparent_tf_returns_background(orc):
    v = W.phantom_small(1)
    tf = orc.TF(const_tf(256, (1, 0.5, 0.25), 0.0), 0, 255)
    bg = (0.1, 0.2, 0.3, 0.4)
    for cam in [W.ortho_camera_small()] + W.orbit_cameras((64, 64, 32), (1, 1, 2), 3):
        r = orc.render(orc.Volume(v, (1, 1, 2)), tf, cam, 40, 30, 0.5, 0.99, bg=bg)
        assert (r.image == np.array(bg)).all()


def test_mirror_symmetric_phantom(orc):
    """The x-symmetric phantom seen from a camera on its symmetry plane gives
    a column-flip symmetric image."""
    v = W.phantom_small_symmetric(1)
    assert (v == v[:, :, ::-1]).all()
    vol = orc.Volume(v, (1, 1, 2))
    tf = orc.TF(W.random_tf(256, 2), 0, 255)
    c = W.box_center((64, 64, 32), (1, 1, 2))
    cams = [W.ortho_camera_small(),
            Camera(tuple(c + [0, -150, 40]), tuple(c), (0, 0, 1), True, 40.0)]
    for cam in cams:
        r = orc.render(vol, tf, cam, 64, 48, 0.5, 0.99)
        np.testing.assert_allclose(r.image, r.image[:, ::-1], atol=1e-12)


def test_axis_permutation_invariance(orc):
    """Swapping the volume's x and y axes and the camera's x and y
    coordinates (and mirroring the image, since the swap flips handedness)
    gives the same picture."""
    v = W.phantom_small(1)
    sp = (1.0, 1.5, 2.0)
    vol = orc.Volume(v, sp)
    volT = orc.Volume(np.ascontiguousarray(v.transpose(0, 2, 1)), (sp[1], sp[0], sp[2]))
    tf = orc.TF(W.random_tf(256, 2), 0, 255)
    sw = lambda p: (p[1], p[0], p[2])
    for cam in W.orbit_cameras((64, 64, 32), sp, 3, elevation_deg=20):
        camT = Camera(sw(cam.eye), sw(cam.center), sw(cam.up), True, cam.fovy_deg)
        a = orc.render(vol, tf, cam, 40, 40, 0.5, 0.99).image
        b = orc.render(volT, tf, camT, 40, 40, 0.5, 0.99).image
        np.testing.assert_allclose(a, b[:, ::-1], atol=1e-9)


def test_linear_in_tf_colour(orc):
    v = W.phantom_small(1)
    vol = orc.Volume(v, (1, 1, 2))
    t = W.random_tf(256, 2)
    t2 = t.copy()
    t2[:, :3] *= np.float32(0.5)
    cam = W.orbit_cameras((64, 64, 32), (1, 1, 2), 2)[1]
    a = orc.render(vol, orc.TF(t, 0, 255), cam, 40, 40, 0.5, 0.99).image
    b = orc.render(vol, orc.TF(t2, 0, 255), cam, 40, 40, 0.5, 0.99).image
    np.testing.assert_allclose(b[..., :3], 0.5 * a[..., :3], atol=1e-12)
    np.testing.assert_allclose(b[..., 3], a[..., 3], atol=0)


def test_pixel_subset_matches_full_image(orc):
    v = W.phantom_small(1)
    vol = orc.Volume(v, (1, 1, 2))
    tf = orc.TF(W.random_tf(256, 2), 0, 255)
    cam = W.orbit_cameras((64, 64, 32), (1, 1, 2), 2)[1]
    full = orc.render(vol, tf, cam, 50, 30, 0.5, 0.99)
    px = np.array([0, 7, 777, 1499, 1000])
    sub = orc.render(vol, tf, cam, 50, 30, 0.5, 0.99, pixels=px)
    np.testing.assert_array_equal(sub.image, full.image.reshape(-1, 4)[px])
    np.testing.assert_array_equal(sub.counts, full.counts.reshape(-1)[px])


# ---------------------------------------------------------------------------
# 8-bit per-brick scaled code
# ---------------------------------------------------------------------------
def test_u8_brick_code(orc):
    rng = np.random.default_rng(21)
    v = rng.integers(0, 4096, size=(19, 23, 34)).astype(np.uint16)
    v[:8, :8, :8] = 77  # a constant brick
    B = 8
    lo, sc, codes = orc.encode_u8_bricks(v, B)
    total, nb = orc.u8_brick_count((34, 23, 19), B)
    assert nb == (5, 3, 3) and total == 45
    f = v.astype(np.float64)
    for bz in range(nb[2]):
        for by in range(nb[1]):
            for bx in range(nb[0]):
                bid = (bz * nb[1] + by) * nb[0] + bx
                blk = f[bz * B:bz * B + B + 1, by * B:by * B + B + 1, bx * B:bx * B + B + 1]
                assert lo[bid] == blk.min()
                hi = blk.max()
                if hi == blk.min():
                    assert sc[bid] == 1.0 and (codes[bid] == 0).all()
                    continue
                assert sc[bid] == np.float32(np.float32(hi) - np.float32(blk.min())) / np.float32(255)
                c = codes[bid].reshape(B + 1, B + 1, B + 1)[:blk.shape[0], :blk.shape[1], :blk.shape[2]]
                dec = lo[bid] + c.astype(np.float64) * sc[bid]
                # half a quantisation step, plus the binary32 rounding of the
                # quotient (v-lo)/scale (code <= 255, relative error <= 2^-23)
                assert np.abs(dec - blk).max() <= sc[bid] * (0.5 + 256 * 2.0 ** -23)
                assert c.min() == 0 and c.max() == 255


def test_u8_brick_owner_rule(orc):
    """A sample is decoded with the brick that owns its cell: at a node shared
    by two bricks, approaching from either side gives that brick's decoding."""
    rng = np.random.default_rng(22)
    v = rng.integers(0, 4096, size=(9, 9, 17)).astype(np.uint16)
    B = 8
    vol = orc.Volume.from_u8_bricks(v, (1, 1, 1), B)
    lo, sc, codes = vol.lo, vol.scale, vol.codes
    # node x=8 is the high halo of brick 0 and the first node of brick 1
    dec0 = lo[0] + codes[0].reshape(9, 9, 9)[3, 4, 8] * np.float64(sc[0])
    dec1 = lo[1] + codes[1].reshape(9, 9, 9)[3, 4, 0] * np.float64(sc[1])
    assert orc.trilinear(vol, [8.0 - 1e-12, 4.0, 3.0]) == pytest.approx(dec0, abs=1e-6)
    assert orc.trilinear(vol, [8.0, 4.0, 3.0]) == pytest.approx(dec1, abs=1e-9)
    # the last node of the volume is reached through the last brick
    dec_last = lo[1] + codes[1].reshape(9, 9, 9)[8, 8, 8] * np.float64(sc[1])
    assert orc.trilinear(vol, [16.0, 8.0, 8.0]) == pytest.approx(dec_last, abs=1e-9)
