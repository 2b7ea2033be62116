"""Thresholding and iso-surface ray functions on the GPU (through the C ABI)
against the FP64 oracle, element by element.

Tolerance: max-abs RGBA error 1e-5 against the oracle's band.  Thresholding
composites with early termination, so the early-termination tie band applies
as for compositing.  A sample whose value lies within 2^-20 of its cell's
largest corner magnitude of a window edge or of the iso-value is decided by
rounding (oracle tie bit 3); the grazing and lattice cases of the projections
(bits 1, 2) change an iso image the same way.  Those pixels are counted and
left out of the comparison.  For the iso-surface the oracle's band spans the
shade over the rounding of the hit refinement and of the six central-
difference values (a weak gradient makes the normal ill-conditioned); every
other pixel must lie within 1e-5 of it and its sample count must match.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-5
DELTA = 1e-6


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1211_5595_amd as rt
    rt.lib()
    return rt


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


def gpu_render(rt, torch, vol, tf, cam, W_, H_, step, fn, lo, hi=0.0, cutoff=0.99, bg=(0, 0, 0, 0), skip=False):
    counts = torch.zeros((H_, W_), dtype=torch.int32, device="cuda")
    img = rt.render(vol, tf, cam, W_, H_, step, cutoff, bg, pixel_counts=counts, ray_function=fn, iso_value=lo,
                    iso_high=hi, skip_empty=skip)
    torch.cuda.synchronize()
    return img.cpu().numpy().astype(np.float64), counts.cpu().numpy()


def check(got, counts, ref, what, max_frac=1 / 500):
    exempt = (ref.tie & (2 | 4 | 8)) != 0
    keep = ~exempt
    dist = np.maximum(np.maximum(ref.band_lo - got, got - ref.band_hi), 0.0).max(-1)
    worst = float(dist[keep].max()) if keep.any() else 0.0
    assert worst <= TOL, f"{what}: distance to the oracle band {worst:.3g} ({exempt.sum()} exempt pixels)"
    exact = keep & ((ref.tie & 1) == 0)
    mism = int((counts != ref.counts)[exact].sum())
    assert mism == 0, f"{what}: {mism} sample counts differ"
    assert exempt.sum() <= max(4, int(exempt.size * max_frac)), f"{what}: {exempt.sum()} rounding-decided pixels"
    return worst, int(exempt.sum())


@pytest.fixture(scope="module")
def small(rt, orc):
    v = W.phantom_small(1)
    return dict(np=v, gv=rt.Volume(v, (1, 1, 2), storage=rt.U8), ov=orc.Volume(v, (1, 1, 2)),
                tf=W.random_tf(256, 2, alpha_max=0.5))


@pytest.fixture(scope="module")
def brain(rt, orc):
    dims, sp = (256, 256, 160), (0.9, 0.9, 1.2)
    v = W.phantom_brain(11)
    return dict(np=v, dims=dims, sp=sp, gv=rt.Volume(v, sp, storage=rt.U16), ov=orc.Volume(v, sp),
                cams=W.orbit_cameras(dims, sp, 36), tf=W.random_tf(4096, 12, alpha_max=0.05))


@pytest.mark.parametrize("fn,lo,hi", [("THRESHOLD", 100.0, 230.0), ("THRESHOLD", 30.0, 120.0), ("ISO", 150.0, 0.0),
                                      ("ISO", 90.0, 0.0)])
def test_small_ortho_full_image(rt, torch_mod, orc, small, fn, lo, hi):
    cam = W.ortho_camera_small()
    got, c = gpu_render(rt, torch_mod, small["gv"], rt.TransferFunction(small["tf"], 0, 255), cam, 128, 128, 0.45,
                        getattr(rt, fn), lo, hi, bg=(0.05, 0.1, 0.15, 0.2))
    ref = orc.render(small["ov"], orc.TF(small["tf"], 0, 255), cam, 128, 128, 0.45, 0.99, bg=(0.05, 0.1, 0.15, 0.2),
                     ray_function=getattr(orc, fn), iso_value=lo, iso_high=hi, tie_delta=DELTA, want_band=True)
    w, n = check(got, c, ref, f"small {fn} {lo}")
    print(f"small {fn} [{lo}, {hi}]: band distance {w:.3g}, exempt {n}")


@pytest.mark.parametrize("fn,lo,hi,view", [("THRESHOLD", 1200.0, 2600.0, 3), ("THRESHOLD", 800.0, 1000.0, 21),
                                           ("ISO", 1000.0, 0.0, 8), ("ISO", 2000.0, 0.0, 27)])
def test_brain_view_full_image(rt, torch_mod, orc, brain, fn, lo, hi, view):
    cam = brain["cams"][view]
    got, c = gpu_render(rt, torch_mod, brain["gv"], rt.TransferFunction(brain["tf"], 0, 4095), cam, 512, 512, 0.5,
                        getattr(rt, fn), lo, hi)
    ref = orc.render(brain["ov"], orc.TF(brain["tf"], 0, 4095), cam, 512, 512, 0.5, 0.99,
                     ray_function=getattr(orc, fn), iso_value=lo, iso_high=hi, tie_delta=DELTA, want_band=True)
    w, n = check(got, c, ref, f"brain {fn} {lo}")
    print(f"brain view {view} {fn} [{lo}, {hi}]: band distance {w:.3g}, exempt {n}, samples {c.sum()}")


@pytest.mark.parametrize("seed", range(8))
def test_random_small_cases(rt, torch_mod, orc, seed):
    rng = np.random.default_rng(700 + seed)
    dims = tuple(int(x) for x in rng.integers(3, 40, 3))
    sp = tuple(float(x) for x in rng.uniform(0.5, 2.0, 3))
    v = rng.integers(0, 4096, size=dims[::-1], dtype=np.uint16)
    v = ((v.astype(np.int64) + np.roll(v, 1, 0) + np.roll(v, 1, 1) + np.roll(v, 1, 2)) // 4).astype(np.uint16)
    fn = ("THRESHOLD", "ISO")[seed % 2]
    lo = float(rng.uniform(800, 2400))
    hi = lo + float(rng.uniform(100, 1500))
    t = W.random_tf(512, seed + 80, alpha_max=0.4)
    cam = W.random_camera(rng, dims, sp)
    Wd, Hd, step = int(rng.integers(1, 80)), int(rng.integers(1, 60)), float(rng.uniform(0.3, 1.1))
    got, c = gpu_render(rt, torch_mod, rt.Volume(v, sp, storage=rt.U16), rt.TransferFunction(t, 0, 4095), cam, Wd,
                        Hd, step, getattr(rt, fn), lo, hi, cutoff=0.95)
    ref = orc.render(orc.Volume(v, sp), orc.TF(t, 0, 4095), cam, Wd, Hd, step, 0.95, ray_function=getattr(orc, fn),
                     iso_value=lo, iso_high=hi, tie_delta=DELTA, want_band=True)
    check(got, c, ref, f"random {seed} {fn} dims {dims}", max_frac=1 / 50)


@pytest.mark.parametrize("storage", ["F32", "F16", "U8_BRICKSCALED", "U15", "U12"])
def test_storage_types(rt, torch_mod, orc, brain, storage):
    v, sp = brain["np"], brain["sp"]
    cam = brain["cams"][12]
    if storage == "F32":
        gv, field = rt.Volume(v, sp, storage=rt.F32), orc.Volume(v.astype(np.float64), sp)
    elif storage == "F16":
        gv, field = rt.Volume(v, sp, storage=rt.F16), orc.Volume(v.astype(np.float16).astype(np.float64), sp)
    elif storage in ("U15", "U12"):  # exact for the 12-bit phantom
        gv, field = rt.Volume(v, sp, storage=getattr(rt, storage)), orc.Volume(v, sp)
    else:
        gv, field = rt.Volume(v, sp, storage=rt.U8_BRICKSCALED, brick=16), orc.Volume.from_u8_bricks(v, sp, 16)
    for fn, lo, hi in (("THRESHOLD", 1200.0, 2600.0), ("ISO", 1000.0, 0.0)):
        got, c = gpu_render(rt, torch_mod, gv, rt.TransferFunction(brain["tf"], 0, 4095), cam, 200, 160, 0.5,
                            getattr(rt, fn), lo, hi)
        ref = orc.render(field, orc.TF(brain["tf"], 0, 4095), cam, 200, 160, 0.5, 0.99,
                         ray_function=getattr(orc, fn), iso_value=lo, iso_high=hi, tie_delta=DELTA, want_band=True)
        check(got, c, ref, f"{storage} {fn}")


def test_threshold_with_skipping_is_bitwise_identical(rt, torch_mod, brain):
    for view, (lo, hi) in ((2, (1200.0, 2600.0)), (17, (300.0, 1600.0))):
        cam = brain["cams"][view]
        tf = rt.TransferFunction(brain["tf"], 0, 4095)
        a, ca = gpu_render(rt, torch_mod, brain["gv"], tf, cam, 256, 256, 0.5, rt.THRESHOLD, lo, hi)
        b, cb = gpu_render(rt, torch_mod, brain["gv"], tf, cam, 256, 256, 0.5, rt.THRESHOLD, lo, hi, skip=True)
        assert np.array_equal(a, b) and np.array_equal(ca, cb)


def test_mixed_batch_bitwise_equal_plain(rt, torch_mod, brain):
    torch = torch_mod
    tf = rt.TransferFunction(brain["tf"], 0, 4095)
    specs = [(rt.ISO, 1000.0, 0.0), (rt.THRESHOLD, 1200.0, 2600.0), (rt.COMPOSITE, 0.0, 0.0), (rt.ISO, 2000.0, 0.0),
             (rt.MIP, 0.0, 0.0), (rt.THRESHOLD, 800.0, 1000.0)]
    jobs = [rt.Job(brain["gv"], tf, brain["cams"][5 * k], 100 + 20 * k, 90 + 12 * k, 0.5, 0.99, ray_function=fn,
                   iso_value=lo, iso_high=hi, skip_empty=(k % 2 == 1)) for k, (fn, lo, hi) in enumerate(specs)]
    plain = [rt.render(brain["gv"], tf, j.camera, j.width, j.height, 0.5, 0.99, ray_function=j.ray_function,
                       iso_value=j.iso_value, iso_high=j.iso_high) for j in jobs]
    outs = rt.render_batch(jobs)
    torch.cuda.synchronize()
    for a, b in zip(plain, outs):
        assert torch.equal(a, b)


def test_invalid_window_and_iso(rt, torch_mod, small):
    out = torch_mod.empty((8, 8, 4), dtype=torch_mod.float32, device="cuda")
    tf = rt.TransferFunction(small["tf"], 0, 255)
    cam = W.ortho_camera_small()
    for opts in (rt.make_opts(ray_function=rt.THRESHOLD, iso_value=5.0, iso_high=4.0),
                 rt.make_opts(ray_function=rt.THRESHOLD, iso_value=float("nan"), iso_high=4.0),
                 rt.make_opts(ray_function=rt.ISO, iso_value=float("inf"))):
        with pytest.raises(rt.InvalidArgument):
            rt.rt_render(small["gv"].handle, small["gv"].dims, None, tf.handle, cam, 8, 8, 0.5, 0.99, None,
                         out.data_ptr(), opts)
