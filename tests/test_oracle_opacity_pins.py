"""Pins of the oracle's optional opacity correction (reading R24): table
opacities are per unit distance u and a sample standing for dt of ray uses
a' = 1 - (1 - a)^(dt/u), applied to the table entries before interpolation.

The pins come from what the correction is for: the opacity of a uniform slab
must depend on its thickness alone, not on the sampling step (closed form
1 - (1-a)^(L/u) for every step, the partial last sample included); with
u = dt the render is the uncorrected one; entry-wise correction differs from
correcting the interpolated opacity (a two-entry table distinguishes them);
ray functions that do not composite per sample are unaffected.
"""
import numpy as np
import pytest

import workloads as W
from workloads import Camera

SLAB_CAM = Camera((1.5, 1.5, -10.0), (1.5, 1.5, 0.0), (0, 1, 0), False, 0.0, 1.0)


def const_tf(K, rgb, a):
    t = np.zeros((K, 4), dtype=np.float32)
    t[:, :3] = np.asarray(rgb, dtype=np.float32)
    t[:, 3] = np.float32(a)
    return t


@pytest.mark.parametrize("step", [0.3, 0.5, 0.7, 1.1, 0.25])
@pytest.mark.parametrize("a,u", [(0.1, 1.5), (0.02, 0.4), (0.5, 3.0)])
def test_slab_opacity_depends_on_thickness_only(orc, step, a, u):
    """Chord L = 3 mm through a uniform 4^3 volume: A = 1-(1-a)^(L/u) at any step."""
    vol = orc.Volume(np.full((4, 4, 4), 7.0), (1, 1, 1))
    c = (0.2, 0.5, 0.9)
    r = orc.render(vol, orc.TF(const_tf(8, c, a), 0, 10), SLAB_CAM, 2, 2, step, 1.0, opacity_unit=u)
    a32 = float(np.float32(a))
    A = 1 - (1 - a32) ** (3.0 / u)
    np.testing.assert_allclose(r.image[..., 3], A, atol=1e-12)
    for ch in range(3):
        np.testing.assert_allclose(r.image[..., ch], float(np.float32(c[ch])) * A, atol=1e-12)


def test_unit_equal_to_dt_is_the_uncorrected_render(orc):
    v = W.phantom_small(1)
    vol = orc.Volume(v, (1, 1, 2))
    tf = orc.TF(W.random_tf(256, 2, alpha_max=0.5), 0, 255)
    cam = W.ortho_camera_small()
    step = 0.45                          # dt = 0.45 * min spacing = 0.45 mm
    plain = orc.render(vol, tf, cam, 48, 48, step, 0.99)
    corr = orc.render(vol, tf, cam, 48, 48, step, 0.99, opacity_unit=0.45)
    np.testing.assert_allclose(corr.image, plain.image, atol=1e-13)
    assert np.array_equal(corr.counts, plain.counts)


def test_correction_is_applied_to_the_entries(orc):
    """Two-entry table, every sample at x = 1/2: the sample opacity is the mean
    of the corrected entries, not the corrected mean."""
    vol = orc.Volume(np.full((4, 4, 4), 5.0), (1, 1, 1))
    t = const_tf(2, (0.3, 0.3, 0.3), 0.0)
    t[0, 3], t[1, 3] = np.float32(0.05), np.float32(0.6)
    step, u = 0.5, 2.0
    r = orc.render(vol, orc.TF(t, 0, 10), SLAB_CAM, 2, 2, step, 1.0, opacity_unit=u)
    q = step / u
    a0, a1 = float(t[0, 3]), float(t[1, 3])
    a_s = 0.5 * ((1 - (1 - a0) ** q) + (1 - (1 - a1) ** q))
    A = 1 - (1 - a_s) ** (3.0 / step)
    np.testing.assert_allclose(r.image[..., 3], A, atol=1e-12)
    wrong = 1 - (1 - 0.5 * (a0 + a1)) ** (3.0 / u)
    assert abs(A - wrong) > 1e-3


def test_projections_and_iso_ignore_it(orc):
    v = W.phantom_small(1)
    vol = orc.Volume(v, (1, 1, 2))
    tf = orc.TF(W.random_tf(256, 2, alpha_max=0.5), 0, 255)
    cam = W.ortho_camera_small()
    for fn, lo in ((orc.MIP, 0.0), (orc.XRAY, 0.0), (orc.AVERAGE, 0.0), (orc.ISO, 120.0)):
        a = orc.render(vol, tf, cam, 32, 32, 0.5, 0.99, ray_function=fn, iso_value=lo)
        b = orc.render(vol, tf, cam, 32, 32, 0.5, 0.99, ray_function=fn, iso_value=lo, opacity_unit=0.3)
        assert np.array_equal(a.image, b.image)


def test_invalid_unit_rejected(orc):
    vol = orc.Volume(np.full((4, 4, 4), 7.0), (1, 1, 1))
    tf = orc.TF(const_tf(8, (1, 1, 1), 0.1), 0, 10)
    for u in (-1.0, float("inf"), float("nan")):
        with pytest.raises(ValueError):
            orc.render(vol, tf, SLAB_CAM, 2, 2, 0.5, 1.0, opacity_unit=u)
