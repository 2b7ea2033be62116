"""Maximum-intensity, X-ray and average-intensity projections on the GPU
(through the C ABI) against the FP64 oracle, element by element.

Tolerance: max-abs RGBA error 1e-5, as for compositing.  A projection has no
early termination, but two rounding-decided cases make both images correct:
a lattice whose last segment is within 1e-6 of empty or full (the maximum
takes the partial sample whatever its weight) and a ray that grazes the box
(hit or miss).  The oracle flags both (tie bits 1 and 2); those pixels are
counted and left out of the value comparison, every other pixel is compared
and its sample count must match exactly.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-5
PROJ = ("MIP", "XRAY", "AVERAGE")


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


def gpu_render(rt, torch, vol, tf, cam, W_, H_, step, rf, bg=(0, 0, 0, 0)):
    counts = torch.zeros((H_, W_), dtype=torch.int32, device="cuda")
    counter = torch.zeros(1, dtype=torch.int64, device="cuda")
    img = rt.render(vol, tf, cam, W_, H_, step, 0.99, bg, pixel_counts=counts, sample_counter=counter,
                    ray_function=getattr(rt, rf))
    torch.cuda.synchronize()
    c = counts.cpu().numpy()
    assert int(counter.item()) == int(c.astype(np.int64).sum())
    return img.cpu().numpy().astype(np.float64), c


def check(got, counts, ref, what):
    exempt = (ref.tie & 6) != 0
    keep = ~exempt
    err = float(np.abs(got - ref.image)[keep].max()) if keep.any() else 0.0
    bad = int((np.abs(got - ref.image).max(-1) > TOL)[keep].sum())
    assert err <= TOL, f"{what}: max abs err {err:.3g} on {bad} pixels ({exempt.sum()} exempt)"
    mism = int((counts != ref.counts)[keep].sum())
    assert mism == 0, f"{what}: {mism} sample counts differ"
    assert exempt.sum() <= max(4, exempt.size // 2000), f"{what}: {exempt.sum()} rounding-decided pixels"
    return err


def window(rf, vmax, chord):
    return (0.0, vmax * chord) if rf == "XRAY" else (0.0, vmax)


@pytest.mark.parametrize("rf", PROJ)
def test_small_ortho_full_image(rt, torch_mod, orc, rf):
    v = W.phantom_small(1)
    t = W.random_tf(256, 2)
    lo, hi = window(rf, 255.0, 40.0)
    gv, gtf = rt.Volume(v, (1, 1, 2), storage=rt.U8), rt.TransferFunction(t, lo, hi)
    cam = W.ortho_camera_small()
    # step 0.45: with 0.5 every axis-parallel chord is a whole number of steps,
    # so every lattice would be decided by rounding
    got, c = gpu_render(rt, torch_mod, gv, gtf, cam, 128, 128, 0.45, rf, bg=(0.1, 0.2, 0.3, 0.4))
    ref = orc.render(orc.Volume(v, (1, 1, 2)), orc.TF(t, lo, hi), cam, 128, 128, 0.45, 0.99,
                     bg=(0.1, 0.2, 0.3, 0.4), ray_function=getattr(orc, rf))
    e = check(got, c, ref, f"small {rf}")
    print(f"small ortho {rf}: max err {e:.3g}")


@pytest.fixture(scope="module")
def brain(rt, orc):
    dims, sp = (256, 256, 160), (0.9, 0.9, 1.2)
    v = W.phantom_brain(11)
    return dict(np=v, dims=dims, sp=sp, gv=rt.Volume(v, sp, storage=rt.U16), ov=orc.Volume(v, sp),
                cams=W.orbit_cameras(dims, sp, 36), tf=W.random_tf(4096, 12, alpha_max=0.6))


@pytest.mark.parametrize("rf", PROJ)
def test_brain_view_full_image(rt, torch_mod, orc, brain, rf):
    lo, hi = window(rf, 4095.0, 150.0)
    cam = brain["cams"][5]
    got, c = gpu_render(rt, torch_mod, brain["gv"], rt.TransferFunction(brain["tf"], lo, hi), cam, 512, 512, 0.5,
                        rf)
    ref = orc.render(brain["ov"], orc.TF(brain["tf"], lo, hi), cam, 512, 512, 0.5, 0.99,
                     ray_function=getattr(orc, rf))
    e = check(got, c, ref, f"brain {rf}")
    print(f"brain 512x512 {rf}: max err {e:.3g}, samples {c.sum()}")


@pytest.mark.parametrize("seed", range(8))
def test_random_small_cases(rt, torch_mod, orc, seed):
    rng = np.random.default_rng(1000 + seed)
    dims = tuple(int(x) for x in rng.integers(2, 48, 3))
    sp = tuple(float(x) for x in rng.uniform(0.4, 2.5, 3))
    v = rng.integers(0, 4096, size=dims[::-1], dtype=np.uint16)
    step = float(rng.uniform(0.2, 1.3))
    Wd, Hd = int(rng.integers(1, 90)), int(rng.integers(1, 70))
    cam = W.random_camera(rng, dims, sp)
    rf = PROJ[seed % 3]
    chord = float(np.sqrt(sum(((n - 1) * s) ** 2 for n, s in zip(dims, sp))))
    lo, hi = window(rf, 4095.0, chord / 2)
    t = W.random_tf(512, seed + 70, alpha_max=0.8)
    got, c = gpu_render(rt, torch_mod, rt.Volume(v, sp, storage=rt.U16), rt.TransferFunction(t, lo, hi), cam,
                        Wd, Hd, step, rf)
    ref = orc.render(orc.Volume(v, sp), orc.TF(t, lo, hi), cam, Wd, Hd, step, 0.99, ray_function=getattr(orc, rf))
    check(got, c, ref, f"random {seed} {rf} dims {dims}")


@pytest.mark.parametrize("storage", ["F32", "F16", "U8_BRICKSCALED", "U15", "U12"])
def test_storage_types(rt, torch_mod, orc, brain, storage):
    """Every sampler variant under the summing projection (the maximum shares
    the sampling code)."""
    v, sp = brain["np"], brain["sp"]
    cam = brain["cams"][17]
    if storage == "F32":
        gv, field = rt.Volume(v, sp, storage=rt.F32), orc.Volume(v.astype(np.float64), sp)
    elif storage == "F16":
        gv, field = rt.Volume(v, sp, storage=rt.F16), orc.Volume(v.astype(np.float16).astype(np.float64), sp)
    elif storage in ("U15", "U12"):  # exact for the 12-bit phantom
        gv, field = rt.Volume(v, sp, storage=getattr(rt, storage)), orc.Volume(v, sp)
    else:
        gv, field = rt.Volume(v, sp, storage=rt.U8_BRICKSCALED, brick=16), orc.Volume.from_u8_bricks(v, sp, 16)
    for rf in ("AVERAGE", "MIP"):
        got, c = gpu_render(rt, torch_mod, gv, rt.TransferFunction(brain["tf"], 0, 4095), cam, 200, 160, 0.5, rf)
        ref = orc.render(field, orc.TF(brain["tf"], 0, 4095), cam, 200, 160, 0.5, 0.99,
                         ray_function=getattr(orc, rf))
        check(got, c, ref, f"{storage} {rf}")


def test_mixed_batch_bitwise_equal_plain(rt, torch_mod, brain):
    """One persistent launch holding compositing and all three projections
    gives each view bit for bit what its own launch gives."""
    torch = torch_mod
    tf_c = rt.TransferFunction(W.random_tf(4096, 12, alpha_max=0.05), 0, 4095)
    tf_p = rt.TransferFunction(brain["tf"], 0, 4095)
    tf_x = rt.TransferFunction(brain["tf"], 0, 4095 * 150.0)
    fns = [("COMPOSITE", tf_c), ("MIP", tf_p), ("XRAY", tf_x), ("AVERAGE", tf_p)] * 2
    specs = [(getattr(rt, f), tf, brain["cams"][4 * k + 1], 96 + 24 * k, 80 + 8 * k) for k, (f, tf) in enumerate(fns)]
    plain = []
    for fn, tf, cam, Wd, Hd in specs:
        plain.append(rt.render(brain["gv"], tf, cam, Wd, Hd, 0.5, 0.99, ray_function=fn))
    jobs = [rt.Job(brain["gv"], tf, cam, Wd, Hd, 0.5, 0.99, ray_function=fn) for fn, tf, cam, Wd, Hd in specs]
    outs = rt.render_batch(jobs)
    plan = rt.BatchPlan(len(jobs), rt.U16)
    jobs2 = [rt.Job(brain["gv"], tf, cam, Wd, Hd, 0.5, 0.99, ray_function=fn) for fn, tf, cam, Wd, Hd in specs]
    plan.launch(jobs2)
    torch.cuda.synchronize()
    for a, b, j in zip(plain, outs, jobs2):
        assert torch.equal(a, b) and torch.equal(a, j.out)


def test_unknown_and_unbuilt_ray_functions(rt, torch_mod):
    v = W.phantom_small(1)
    gv, gtf = rt.Volume(v, (1, 1, 2), storage=rt.U8), rt.TransferFunction(W.random_tf(256, 2), 0, 255)
    out = torch_mod.empty((8, 8, 4), dtype=torch_mod.float32, device="cuda")
    cam = W.ortho_camera_small()
    with pytest.raises(rt.InvalidArgument):
        rt.rt_render(gv.handle, gv.dims, None, gtf.handle, cam, 8, 8, 0.5, 0.99, None, out.data_ptr(),
                     rt.make_opts(ray_function=9))
