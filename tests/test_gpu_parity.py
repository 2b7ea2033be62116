"""GPU path (through the C ABI) against the FP64 oracle, element by element.

Tolerance: max-abs RGBA error 1e-5 on the binary32 path.  Early ray
termination is a threshold on accumulated opacity, so where the binary32 and
binary64 opacities sit within 1e-6 of the cutoff either stopping point is
correct: the oracle reports the per-channel range of all such outputs (its
tie band) and a GPU value passes when it lies inside that range widened by
the tolerance.  Sample counts must match exactly except on pixels the oracle
flags as ties.
"""
import math

import numpy as np
import pytest

import workloads as W
from workloads import Camera

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


def gpu_render(rt, torch, vol, tf, cam, W_, H_, step, cutoff, bg=(0, 0, 0, 0), **kw):
    counts = torch.zeros((H_, W_), dtype=torch.int32, device="cuda")
    counter = torch.zeros(1, dtype=torch.int64, device="cuda")
    img = rt.render(vol, tf, cam, W_, H_, step, cutoff, bg, pixel_counts=counts, sample_counter=counter, **kw)
    torch.cuda.synchronize()
    c = counts.cpu().numpy()
    assert int(counter.item()) == int(c.astype(np.int64).sum())
    return img.cpu().numpy().astype(np.float64), c


def check(got, ref, counts=None, what=""):
    """got: [..., 4] float64 GPU values; ref: oracle result with band."""
    lo, hi = ref.band_lo, ref.band_hi
    dist = np.maximum(np.maximum(lo - got, got - hi), 0.0)
    worst = float(dist.max()) if dist.size else 0.0
    tie = ref.tie != 0
    plain = ~tie
    err_plain = float(np.abs(got - ref.image)[plain].max()) if plain.any() else 0.0
    assert worst <= TOL, f"{what}: max distance to the oracle's tie band {worst:.3g} (max abs err off ties {err_plain:.3g})"
    assert err_plain <= TOL, f"{what}: max abs err {err_plain:.3g}"
    if counts is not None:
        et_tie = (ref.tie & 1) != 0
        lat_tie = (ref.tie & 6) != 0
        exact = ~(et_tie | lat_tie)
        mism = (counts != ref.counts) & exact
        assert not mism.any(), f"{what}: {mism.sum()} sample counts differ off ties"
        assert (np.abs(counts - ref.counts)[lat_tie & ~et_tie] <= 1).all()
    return worst, err_plain


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def small(rt, orc):
    v = W.phantom_small(1)
    t = W.random_tf(256, 2)
    return dict(np=v, tf_np=t, gv=rt.Volume(v, (1, 1, 2), storage=rt.U8), gtf=rt.TransferFunction(t, 0, 255),
                ov=orc.Volume(v, (1, 1, 2)), otf=orc.TF(t, 0, 255))


@pytest.fixture(scope="module")
def brain(rt, orc):
    dims, sp = (256, 256, 160), (0.9, 0.9, 1.2)
    v = W.phantom_brain(11)
    t = W.random_tf(4096, 12, alpha_max=0.05)
    return dict(np=v, tf_np=t, dims=dims, sp=sp, gv=rt.Volume(v, sp, storage=rt.U16),
                gtf=rt.TransferFunction(t, 0, 4095), ov=orc.Volume(v, sp), otf=orc.TF(t, 0, 4095),
                cams=W.orbit_cameras(dims, sp, 36))


def test_small_ortho_full_image(rt, torch_mod, orc, small):
    cam = W.ortho_camera_small()
    got, c = gpu_render(rt, torch_mod, small["gv"], small["gtf"], cam, 128, 128, 0.5, 0.99)
    ref = orc.render(small["ov"], small["otf"], cam, 128, 128, 0.5, 0.99, tie_delta=DELTA, want_band=True)
    w, e = check(got, ref, c, "small ortho")
    print(f"small ortho 128x128: max err {e:.3g}, band dist {w:.3g}, ties {(ref.tie & 1).sum()}")


@pytest.mark.parametrize("view", [0, 9, 22, 31])
def test_brain_views_full_image(rt, torch_mod, orc, brain, view):
    cam = brain["cams"][view]
    got, c = gpu_render(rt, torch_mod, brain["gv"], brain["gtf"], cam, 512, 512, 0.5, 0.99)
    ref = orc.render(brain["ov"], brain["otf"], cam, 512, 512, 0.5, 0.99, tie_delta=DELTA, want_band=True)
    w, e = check(got, ref, c, f"brain view {view}")
    print(f"brain view {view} 512x512: max err {e:.3g}, band dist {w:.3g}, ties {(ref.tie & 1).sum()}, "
          f"samples {c.sum()}")


def test_brain_orbit_sampled(rt, torch_mod, orc, brain):
    """All 36 orbit views at full size, 2048 pixels each checked one by one."""
    rng = np.random.default_rng(77)
    worst = 0.0
    for vi, cam in enumerate(brain["cams"]):
        got, c = gpu_render(rt, torch_mod, brain["gv"], brain["gtf"], cam, 512, 512, 0.5, 0.99)
        px = rng.choice(512 * 512, size=2048, replace=False)
        ref = orc.render(brain["ov"], brain["otf"], cam, 512, 512, 0.5, 0.99, pixels=px, tie_delta=DELTA,
                         want_band=True)
        w, _ = check(got.reshape(-1, 4)[px], ref, c.reshape(-1)[px], f"brain view {vi}")
        worst = max(worst, w)
    print(f"36 views sampled: worst band distance {worst:.3g}")


# ---------------------------------------------------------------------------
# ragged, degenerate and random cases
# ---------------------------------------------------------------------------
def _random_case(seed):
    rng = np.random.default_rng(seed)
    dims = tuple(int(x) for x in rng.integers(2, 40, size=3))
    sp = tuple(float(x) for x in rng.uniform(0.3, 2.5, size=3))
    v = rng.integers(0, 4096, size=dims[::-1]).astype(np.uint16)
    if seed % 3 == 0:  # smooth content as well as noise
        v = W.phantom_brain(seed, dims=dims, spacing=sp) if min(dims) > 4 else v
    c = W.box_center(dims, sp)
    R = W.bounding_radius(dims, sp)
    kind = seed % 4
    if kind == 0:      # perspective from outside
        cam = W.random_camera(rng, dims, sp)
    elif kind == 1:    # eye inside the volume
        eye = c + rng.uniform(-0.3, 0.3, 3) * np.array([(n - 1) * s for n, s in zip(dims, sp)])
        cam = Camera(tuple(eye), tuple(eye + rng.normal(size=3)), (0, 0, 1), True, float(rng.uniform(30, 120)))
    elif kind == 2:    # orthographic, oblique
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        cam = Camera(tuple(c - 3 * R * d), tuple(c), (0, 1, 0) if abs(d[1]) < 0.9 else (1, 0, 0), False, 0.0,
                     float(rng.uniform(0.5, 1.5) * R))
    else:              # perspective, close and wide
        cam = Camera(tuple(c + 1.3 * R * np.array([0.3, -1, 0.4])), tuple(c), (0, 0, 1), True, 100.0)
    Wd, Hd = [(1, 1), (7, 13), (65, 33), (130, 67), (64, 64), (3, 200)][seed % 6]
    step = float(rng.uniform(0.3, 1.7))
    cutoff = [0.5, 0.99, 1.0][seed % 3]
    tf = W.random_tf(4096, seed, alpha_max=float(rng.uniform(0.02, 0.6)))
    bg = tuple(float(x) for x in rng.uniform(0, 1, 4)) if seed % 2 else (0, 0, 0, 0)
    return v, dims, sp, cam, Wd, Hd, step, cutoff, tf, bg


@pytest.mark.parametrize("seed", range(24))
def test_random_small_cases(rt, torch_mod, orc, seed):
    v, dims, sp, cam, Wd, Hd, step, cutoff, tf, bg = _random_case(seed)
    gv = rt.Volume(v, sp, storage=rt.U16)
    gtf = rt.TransferFunction(tf, 0, 4095)
    got, c = gpu_render(rt, torch_mod, gv, gtf, cam, Wd, Hd, step, cutoff, bg)
    ref = orc.render(orc.Volume(v, sp), orc.TF(tf, 0, 4095), cam, Wd, Hd, step, cutoff, bg=bg, tie_delta=DELTA,
                     want_band=True)
    check(got, ref, c, f"case {seed} dims {dims} {Wd}x{Hd}")


def test_minimal_volume_and_axis_rays(rt, torch_mod, orc):
    """2x2x2 volume; rays exactly parallel to the axes (zero direction
    components) through a 4x4 orthographic image and a perspective one."""
    v = np.array([[[0, 4095], [1000, 3000]], [[2000, 500], [4095, 100]]], dtype=np.uint16)
    tf = W.random_tf(4096, 5, alpha_max=0.8)
    gv, gtf = rt.Volume(v, (1, 1, 1), storage=rt.U16), rt.TransferFunction(tf, 0, 4095)
    ov, otf = orc.Volume(v, (1, 1, 1)), orc.TF(tf, 0, 4095)
    cams = [Camera((0.5, 0.5, -5), (0.5, 0.5, 0), (0, 1, 0), False, 0.0, 0.4),
            Camera((0.5, 7, 0.5), (0.5, 0, 0.5), (0, 0, 1), False, 0.0, 0.45),
            Camera((0.5, 0.5, 6), (0.5, 0.5, 0.5), (0, 1, 0), True, 20.0)]
    for cam in cams:
        for step in (0.25, 0.3, 1.0):
            got, c = gpu_render(rt, torch_mod, gv, gtf, cam, 4, 4, step, 1.0)
            ref = orc.render(ov, otf, cam, 4, 4, step, 1.0, tie_delta=DELTA, want_band=True)
            check(got, ref, c, f"2x2x2 {cam} step {step}")


def test_transparent_tf_gives_background_exactly(rt, torch_mod, small):
    tf0 = rt.TransferFunction(np.zeros((256, 4), np.float32), 0, 255)
    bg = (0.25, 0.5, 0.125, 0.75)
    for cam in [W.ortho_camera_small()] + W.orbit_cameras((64, 64, 32), (1, 1, 2), 4):
        got, _ = gpu_render(rt, torch_mod, small["gv"], tf0, cam, 70, 50, 0.5, 0.99, bg)
        assert (got == np.array(bg, dtype=np.float32)).all()


def test_tile_shapes_and_workgroups_bitwise(rt, torch_mod, brain):
    cam = brain["cams"][5]
    base, _ = gpu_render(rt, torch_mod, brain["gv"], brain["gtf"], cam, 300, 200, 0.5, 0.99)
    for tile, waves in [((16, 4), 16), ((4, 16), 8), ((32, 2), 4), ((8, 8), 1), ((64, 1), 2)]:
        got, _ = gpu_render(rt, torch_mod, brain["gv"], brain["gtf"], cam, 300, 200, 0.5, 0.99, tile=tile,
                            waves_per_block=waves)
        assert np.array_equal(got, base), (tile, waves)


# ---------------------------------------------------------------------------
# storage types: binary32, half, per-brick 8-bit
# ---------------------------------------------------------------------------
def test_f32_and_f16_storage(rt, torch_mod, orc, brain):
    v = brain["np"]
    cam = brain["cams"][3]
    for storage, field in [(rt.F32, v.astype(np.float64)),
                           (rt.F16, v.astype(np.float16).astype(np.float64))]:
        gv = rt.Volume(v, brain["sp"], storage=storage)
        got, c = gpu_render(rt, torch_mod, gv, brain["gtf"], cam, 256, 256, 0.5, 0.99)
        ref = orc.render(orc.Volume(field, brain["sp"]), brain["otf"], cam, 256, 256, 0.5, 0.99,
                         tie_delta=DELTA, want_band=True)
        check(got, ref, c, f"storage {storage}")


@pytest.mark.parametrize("storage", ["U8", "U16", "F16", "F32"])
def test_linear_and_cell_layouts_bitwise_equal(rt, torch_mod, storage):
    """Both layouts hold the same corner values and the marcher blends them
    in the same order, so the images agree bit for bit."""
    v = W.phantom_brain(5, dims=(61, 47, 38))
    if storage == "U8":
        v = (v >> 4).astype(np.uint8)
    st = getattr(rt, storage)
    imgs = []
    for layout in (rt.LAYOUT_CELLS, rt.LAYOUT_LINEAR):
        gv = rt.Volume(v, (0.9, 0.9, 1.2), storage=st, layout=layout)
        gtf = rt.TransferFunction(W.random_tf(4096, 3, alpha_max=0.1), 0, 4095 if storage != "U8" else 255)
        cam = W.orbit_cameras((61, 47, 38), (0.9, 0.9, 1.2), 7)[3]
        img, c = gpu_render(rt, torch_mod, gv, gtf, cam, 97, 75, 0.5, 0.99)
        imgs.append((img, c))
    assert np.array_equal(imgs[0][0], imgs[1][0]) and np.array_equal(imgs[0][1], imgs[1][1])


def poly_coefficients(v):
    """Trilinear polynomial coefficients of every padded cell (-1..n-1 per
    axis, corners clamped to the grid), in int64."""
    g = np.pad(v.astype(np.int64), 1, mode="edge")             # padded nodes -1..n
    c = {}
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                c[dx, dy, dz] = g[dz: dz + g.shape[0] - 1, dy: dy + g.shape[1] - 1, dx: dx + g.shape[2] - 1]
    p0 = c[0, 0, 0]
    px, py, pz = c[1, 0, 0] - p0, c[0, 1, 0] - p0, c[0, 0, 1] - p0
    pxy = c[1, 1, 0] - c[1, 0, 0] - c[0, 1, 0] + p0
    pxz = c[1, 0, 1] - c[1, 0, 0] - c[0, 0, 1] + p0
    pyz = c[0, 1, 1] - c[0, 1, 0] - c[0, 0, 1] + p0
    pxyz = c[1, 1, 1] - c[1, 1, 0] - c[1, 0, 1] - c[0, 1, 1] + c[1, 0, 0] + c[0, 1, 0] + c[0, 0, 1] - p0
    return np.stack([p0, px, py, pz, pxy, pxz, pyz, pxyz], -1)   # [cz, cy, cx, 8]


@pytest.mark.parametrize("storage", ["U8", "U16"])
def test_poly_layout_coefficients_exact(rt, torch_mod, storage):
    """Every stored coefficient equals the integer combination of the cell's
    corners (all of them are exact in binary32)."""
    dims = (13, 10, 7)
    v = W.phantom_brain(21, dims=dims)
    if storage == "U8":
        v = (v >> 4).astype(np.uint8)
    gv = rt.Volume(v, (0.9, 0.9, 1.2), storage=getattr(rt, storage), layout=rt.LAYOUT_POLY)
    torch_mod.cuda.synchronize()
    nb = [(n + 2) // 2 for n in dims]
    raw = gv.buf.cpu().numpy()[: nb[0] * nb[1] * nb[2] * 8 * 32].view(np.float32)
    blocks = raw.reshape(nb[2], nb[1], nb[0], 2, 2, 2, 8)              # [bz, by, bx, wz, wy, wx, 8]
    cells = blocks.transpose(0, 3, 1, 4, 2, 5, 6).reshape(2 * nb[2], 2 * nb[1], 2 * nb[0], 8)
    want = poly_coefficients(v)                                          # cells -1..n-1 per axis
    got = cells[: dims[2] + 1, : dims[1] + 1, : dims[0] + 1]
    assert np.array_equal(got.astype(np.int64), want) and np.array_equal(got, want.astype(np.float32))


def test_poly_layout_render_parity(rt, torch_mod, orc, small, brain):
    """The polynomial layout evaluates the same trilinear interpolant in a
    different order, so it meets the oracle at the same tolerance."""
    gv = rt.Volume(small["np"], (1, 1, 2), storage=rt.U8, layout=rt.LAYOUT_POLY)
    cam = W.ortho_camera_small()
    got, c = gpu_render(rt, torch_mod, gv, small["gtf"], cam, 128, 128, 0.5, 0.99)
    ref = orc.render(small["ov"], small["otf"], cam, 128, 128, 0.5, 0.99, tie_delta=DELTA, want_band=True)
    check(got, ref, c, "poly small")
    gv = rt.Volume(brain["np"], brain["sp"], storage=rt.U16, layout=rt.LAYOUT_POLY)
    for view in (0, 13):
        cam = brain["cams"][view]
        got, c = gpu_render(rt, torch_mod, gv, brain["gtf"], cam, 512, 512, 0.5, 0.99)
        ref = orc.render(brain["ov"], brain["otf"], cam, 512, 512, 0.5, 0.99, tie_delta=DELTA, want_band=True)
        w, e = check(got, ref, c, f"poly brain view {view}")
        print(f"poly brain view {view}: max err {e:.3g}, band dist {w:.3g}")
    rng = np.random.default_rng(5)
    for seed in range(6):
        dims = tuple(int(x) for x in rng.integers(2, 40, 3))
        sp = tuple(float(x) for x in rng.uniform(0.5, 2.0, 3))
        v = rng.integers(0, 4096, size=dims[::-1], dtype=np.uint16)
        t = W.random_tf(512, seed + 40, alpha_max=0.3)
        cam = W.random_camera(rng, dims, sp)
        gv = rt.Volume(v, sp, storage=rt.U16, layout=rt.LAYOUT_POLY)
        got, c = gpu_render(rt, torch_mod, gv, rt.TransferFunction(t, 0, 4095), cam, 67, 45, 0.37, 0.95)
        ref = orc.render(orc.Volume(v, sp), orc.TF(t, 0, 4095), cam, 67, 45, 0.37, 0.95, tie_delta=DELTA,
                         want_band=True)
        check(got, ref, c, f"poly random {seed} dims {dims}")


def test_poly_layout_batch_equals_plain(rt, torch_mod, brain):
    torch = torch_mod
    gv = rt.Volume(brain["np"], brain["sp"], storage=rt.U16, layout=rt.LAYOUT_POLY)
    cams = brain["cams"][::7]
    plain = [gpu_render(rt, torch, gv, brain["gtf"], c, 160, 128, 0.5, 0.99)[0] for c in cams]
    jobs = [rt.Job(gv, brain["gtf"], c, 160, 128, 0.5, 0.99) for c in cams]
    outs = rt.render_batch(jobs)
    plan = rt.BatchPlan(8, rt.U16, layout=rt.LAYOUT_POLY)
    with pytest.raises(rt.InvalidArgument):  # cells plan, poly volume
        rt.BatchPlan(8, rt.U16).launch(jobs)
    jobs2 = [rt.Job(gv, brain["gtf"], c, 160, 128, 0.5, 0.99) for c in cams]
    plan.launch(jobs2)
    torch.cuda.synchronize()
    for a, b, j in zip(plain, outs, jobs2):
        assert np.array_equal(a, b.cpu().numpy().astype(np.float64))
        assert np.array_equal(a, j.out.cpu().numpy().astype(np.float64))


def test_f16_relayout_rounds_to_nearest_even(rt, torch_mod):
    v = np.arange(0, 4096, dtype=np.uint16)[None, None, :].repeat(2, 0).repeat(2, 1)
    gv = rt.Volume(v, (1, 1, 1), storage=rt.F16, layout=rt.LAYOUT_LINEAR)
    torch_mod.cuda.synchronize()
    raw = gv.buf[: (4098 * 4 * 4) * 2].view(torch_mod.float16).cpu().numpy().reshape(4, 4, 4098)
    want = v[0, 0].astype(np.float16)
    assert np.array_equal(raw[1, 1, 1:-1].view(np.uint16), want.view(np.uint16))
    assert raw[1, 1, 0] == want[0] and raw[1, 1, -1] == want[-1]   # replicated border


@pytest.mark.parametrize("B", [8, 16])
def test_u8_brick_codes_bit_exact(rt, torch_mod, orc, B):
    v = W.phantom_brain(11, dims=(70, 45, 33))
    dims = (70, 45, 33)
    gv = rt.Volume(v, (0.9, 0.9, 1.2), storage=rt.U8_BRICKSCALED, brick=B, layout=rt.LAYOUT_BRICKS)
    torch_mod.cuda.synchronize()
    lo, sc, codes = orc.encode_u8_bricks(v, B)
    total, nb = orc.u8_brick_count(dims, B)
    raw = gv.buf.cpu().numpy()
    par = raw[: total * 8].view(np.float32).reshape(total, 2)
    assert np.array_equal(par[:, 0].view(np.uint32), lo.view(np.uint32))
    assert np.array_equal(par[:, 1].view(np.uint32), sc.view(np.uint32))
    off = ((total * 8 + 255) // 256) * 256
    S = B + 3
    dev = raw[off: off + total * S ** 3].reshape(total, S, S, S)
    ref = codes.reshape(total, B + 1, B + 1, B + 1)
    for bid in range(total):
        bx, by, bz = bid % nb[0], (bid // nb[0]) % nb[1], bid // (nb[0] * nb[1])
        ex = min(B, dims[0] - 1 - bx * B) + 1
        ey = min(B, dims[1] - 1 - by * B) + 1
        ez = min(B, dims[2] - 1 - bz * B) + 1
        assert np.array_equal(dev[bid, 1:1 + ez, 1:1 + ey, 1:1 + ex], ref[bid, :ez, :ey, :ex]), bid


@pytest.mark.parametrize("layout,B", [("LAYOUT_BRICKS", 16), ("LAYOUT_CELLS", 16), ("LAYOUT_CELLS", 8),
                                      ("LAYOUT_CELLS", 32)])
def test_u8_brick_storage_render(rt, torch_mod, orc, brain, layout, B):
    v = brain["np"]
    cam = brain["cams"][7]
    gv = rt.Volume(v, brain["sp"], storage=rt.U8_BRICKSCALED, brick=B, layout=getattr(rt, layout))
    got, c = gpu_render(rt, torch_mod, gv, brain["gtf"], cam, 256, 256, 0.5, 0.99)
    ref = orc.render(orc.Volume.from_u8_bricks(v, brain["sp"], B), brain["otf"], cam, 256, 256, 0.5, 0.99,
                     tie_delta=DELTA, want_band=True)
    check(got, ref, c, f"u8 bricks {layout} B={B}")



@pytest.mark.parametrize("storage", ["F16", "U8_BRICKSCALED"])
def test_precision_orbit_full_size_sampled(rt, torch_mod, orc, brain, storage):
    """The reduced-precision workload at its full size: 8 orbit views of the
    brain phantom at 1024x1024, step 0.25 voxel, in one batch plan, from half
    cells or 8-bit brick codes (B = 16), against the oracle on the stored
    field: views 0 and 3 whole (every pixel), 768 sampled pixels of each of
    the others."""
    torch = torch_mod
    v = brain["np"]
    if storage == "F16":
        gv = rt.Volume(v, brain["sp"], storage=rt.F16)
        ov = orc.Volume(v.astype(np.float16).astype(np.float64), brain["sp"])
    else:
        gv = rt.Volume(v, brain["sp"], storage=rt.U8_BRICKSCALED, brick=16)
        ov = orc.Volume.from_u8_bricks(v, brain["sp"], 16)
    cams = W.orbit_cameras(brain["dims"], brain["sp"], 8)
    pix = [torch.zeros((1024, 1024), dtype=torch.int32, device="cuda") for _ in cams]
    jobs = [rt.Job(gv, brain["gtf"], c, 1024, 1024, 0.25, 0.99, pixel_counts=p) for c, p in zip(cams, pix)]
    rt.BatchPlan(len(jobs), getattr(rt, storage)).launch(jobs)
    torch.cuda.synchronize()
    rng = np.random.default_rng(79)
    for vi, (cam, j, p) in enumerate(zip(cams, jobs, pix)):
        if vi in (0, 3):
            ref = orc.render(ov, brain["otf"], cam, 1024, 1024, 0.25, 0.99, tie_delta=DELTA, want_band=True)
            w, e = check(j.out.cpu().numpy().astype(np.float64), ref, p.cpu().numpy(),
                         f"{storage} 1024x1024 whole view {vi}")
            print(f"{storage} 1024x1024 whole view {vi}: max err {e:.3g}, band distance {w:.3g}, "
                  f"ties {int(((ref.tie & 1) != 0).sum())}")
            continue
        px = rng.choice(1024 * 1024, size=768, replace=False)
        ref = orc.render(ov, brain["otf"], cam, 1024, 1024, 0.25, 0.99, pixels=px, tie_delta=DELTA, want_band=True)
        got = j.out.cpu().numpy().astype(np.float64).reshape(-1, 4)[px]
        check(got, ref, p.cpu().numpy().reshape(-1)[px], f"{storage} 1024x1024 view {vi}")


@pytest.fixture(scope="module")
def largest(rt, orc):
    """The largest grid of the cell layout, 508 x 510 x 510 nodes (255 x 256 x
    256 blocks of 2x2x2 cells, one block short of the 2^24 the layout takes):
    a separable smooth field plus separable integer noise, cheap at 132 M
    nodes, and the oracle's view of it."""
    dims, sp = (508, 510, 510), (1.0, 1.0, 1.0)
    ax = [np.arange(n, dtype=np.float32) for n in dims]
    smooth = (np.sin(ax[2] / 29.0 + 0.5)[:, None, None] * np.cos(ax[1] / 23.0)[None, :, None]
              * (1500.0 * np.sin(ax[0] / 17.0)).astype(np.float32)[None, None, :])
    hrng = np.random.default_rng(81)
    hz, hy, hx = (hrng.integers(0, 81, size=n).astype(np.int16) for n in dims[::-1])
    noise = (hz[:, None, None] + hy[None, :, None]) + hx[None, None, :]
    v = (np.rint(smooth).astype(np.int16) + (noise % 81 - 40) + 2048).astype(np.uint16)
    del smooth, noise
    return dims, sp, v, orc.Volume(v, sp)


@pytest.mark.parametrize("storage", ["U12", "F32"])
def test_largest_cell_volume(rt, torch_mod, orc, largest, storage):
    """Cell offsets of the largest grid reach 2^31 bytes (12-bit cells) and
    2^32 bytes (binary32 cells).  Rays through the far corner, where the
    offsets are largest, and through the whole volume, from one launch and
    from a batch, against the oracle on sampled pixels."""
    torch = torch_mod
    dims, sp, v, ov = largest
    st = getattr(rt, storage)
    assert rt.rt_volume_bytes(dims, st) >= (1 << (32 if storage == "F32" else 31)) - (1 << 26)
    gv = rt.Volume(v, sp, storage=st)
    t = W.random_tf(4096, 33, alpha_max=0.05)
    gtf, otf = rt.TransferFunction(t, 0, 4095), orc.TF(t, 0, 4095)
    hi = np.array([(n - 1) * s for n, s in zip(dims, sp)])
    corner = Camera(tuple(hi + np.array([90.0, 70.0, 60.0])), tuple(hi - 60.0), (0, 0, 1), True, 40.0)
    cams = [corner, W.orbit_cameras(dims, sp, 8)[3]]
    rng = np.random.default_rng(80)
    for ci, cam in enumerate(cams):
        got, c = gpu_render(rt, torch, gv, gtf, cam, 192, 160, 0.5, 0.99)
        out = rt.render_batch([rt.Job(gv, gtf, cam, 192, 160, 0.5, 0.99)])[0]
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().astype(np.float64), got)
        assert (c > 0).mean() > 0.3
        px = rng.choice(192 * 160, size=400, replace=False)
        ref = orc.render(ov, otf, cam, 192, 160, 0.5, 0.99, pixels=px, tie_delta=DELTA, want_band=True)
        check(got.reshape(-1, 4)[px], ref, c.reshape(-1)[px], f"{storage} largest cell volume, camera {ci}")

@pytest.mark.parametrize("B", [8, 16])
def test_u8_brick_cells_codes_bit_exact(rt, torch_mod, orc, B):
    """Every stored cell carries its 8 corner codes from the owning brick's
    encoding and the block carries that brick's (lo, scale), bit for bit."""
    dims = (37, 29, 21)
    v = W.phantom_brain(13, dims=dims)
    gv = rt.Volume(v, (0.9, 0.9, 1.2), storage=rt.U8_BRICKSCALED, brick=B, layout=rt.LAYOUT_CELLS)
    torch_mod.cuda.synchronize()
    lo, sc, codes = orc.encode_u8_bricks(v, B)
    _, nb = orc.u8_brick_count(dims, B)
    ref = codes.reshape(-1, B + 1, B + 1, B + 1)
    cb = [(n + 1) // 2 + 1 for n in dims]
    ncb = cb[0] * cb[1] * cb[2]
    raw = gv.buf.cpu().numpy()
    par = raw[: ncb * 8].view(np.float32).reshape(ncb, 2)
    off = (ncb * 8 + 255) // 256 * 256
    cells = raw[off: off + ncb * 64].reshape(ncb, 8, 8)
    rng = np.random.default_rng(1)
    for _ in range(400):
        c = [int(rng.integers(0, n - 1)) for n in dims]          # an interior cell
        b = [(x + 2) // 2 for x in c]                            # its shifted block
        w = [(x + 2) % 2 for x in c]
        blk = (b[2] * cb[1] + b[1]) * cb[0] + b[0]
        own = [x // B for x in c]
        bid = (own[2] * nb[1] + own[1]) * nb[0] + own[0]
        assert par[blk, 0].view(np.uint32) == lo[bid].view(np.uint32)
        assert par[blk, 1].view(np.uint32) == sc[bid].view(np.uint32)
        got = cells[blk, w[0] | (w[1] << 1) | (w[2] << 2)]
        for k in range(8):
            dx, dy, dz = k & 1, (k >> 1) & 1, k >> 2
            assert got[k] == ref[bid, c[2] - own[2] * B + dz, c[1] - own[1] * B + dy, c[0] - own[0] * B + dx]


# ---------------------------------------------------------------------------
# batching: bitwise identical to the plain per-view launch
# ---------------------------------------------------------------------------
def test_batch_and_plan_bitwise_equal_plain(rt, torch_mod, small, brain):
    torch = torch_mod
    v2 = W.phantom_brain(3, dims=(96, 80, 64))
    gv2 = rt.Volume(v2, (0.9, 0.9, 1.2), storage=rt.U16)
    tf2 = rt.TransferFunction(W.random_tf(1024, 9, alpha_max=0.2), 0, 4095)
    rng = np.random.default_rng(3)
    specs = []
    for k in range(7):
        if k % 2:
            specs.append((brain["gv"], brain["gtf"], brain["cams"][k * 5], 200 + 17 * k, 150 + 9 * k))
        else:
            specs.append((gv2, tf2, W.random_camera(rng, (96, 80, 64), (0.9, 0.9, 1.2)), 64 + 40 * k, 97))
    plain = []
    for vol, tf, cam, Wd, Hd in specs:
        img, _ = gpu_render(rt, torch, vol, tf, cam, Wd, Hd, 0.5, 0.99)
        plain.append(img)
    jobs = [rt.Job(vol, tf, cam, Wd, Hd, 0.5, 0.99) for vol, tf, cam, Wd, Hd in specs]
    counter = torch.zeros(1, dtype=torch.int64, device="cuda")
    outs = rt.render_batch(jobs, sample_counter=counter)
    torch.cuda.synchronize()
    for a, b in zip(plain, outs):
        assert np.array_equal(a, b.cpu().numpy().astype(np.float64))
    n1 = int(counter.item())
    plan = rt.BatchPlan(16, rt.U16)
    with pytest.raises(rt.InvalidArgument):  # plan built for another layout
        rt.BatchPlan(4, rt.U16, layout=rt.LAYOUT_LINEAR).launch(jobs[:1])
    for rep in range(3):  # replays with eager work in between
        for j in jobs:
            j.out.zero_()
        sub = jobs if rep != 1 else jobs[2:5]
        c2 = torch.zeros(1, dtype=torch.int64, device="cuda")
        plan.launch(sub, sample_counter=c2)
        torch.cuda.synchronize()
        ref = plain if rep != 1 else plain[2:5]
        for a, j in zip(ref, sub):
            assert np.array_equal(a, j.out.cpu().numpy().astype(np.float64)), rep
        if rep != 1:
            assert int(c2.item()) == n1



def test_largest_batch_and_widest_images(rt, torch_mod, orc, small):
    """4096 jobs, the most a batch takes (tiny images, random cameras, three
    tables), from a one-off launch and a plan, bitwise equal to one launch per
    view, with the launch-wide counter equal to the per-view counts; and images
    32768 pixels wide or high, the largest side, against the oracle."""
    torch = torch_mod
    rng = np.random.default_rng(82)
    dims, sp = (64, 64, 32), (1, 1, 2)
    tfs = [rt.TransferFunction(W.random_tf(256, 40 + k, alpha_max=0.4), 0, 255) for k in range(3)]
    specs = [(W.random_camera(rng, dims, sp), int(rng.integers(1, 6)), int(rng.integers(1, 5)), k % 3)
             for k in range(4096)]
    pix = [torch.zeros((h, w), dtype=torch.int32, device="cuda") for _, w, h, _ in specs]
    jobs = [rt.Job(small["gv"], tfs[t], cam, w, h, 0.5, 0.99, pixel_counts=p) for (cam, w, h, t), p in zip(specs, pix)]
    counter = torch.zeros(1, dtype=torch.int64, device="cuda")
    rt.render_batch(jobs, sample_counter=counter)
    plan = rt.BatchPlan(4096, rt.U8)
    pj = [rt.Job(small["gv"], tfs[t], cam, w, h, 0.5, 0.99) for cam, w, h, t in specs]
    c2 = torch.zeros(1, dtype=torch.int64, device="cuda")
    plan.launch(pj, sample_counter=c2)
    torch.cuda.synchronize()
    assert int(counter.item()) == sum(int(p.sum()) for p in pix) == int(c2.item())
    assert all(torch.equal(a.out, b.out) for a, b in zip(jobs, pj))
    for k in range(0, 4096, 16):  # one launch per view, every 16th job
        cam, w, h, t = specs[k]
        ref, cnt = gpu_render(rt, torch, small["gv"], tfs[t], cam, w, h, 0.5, 0.99)
        assert np.array_equal(jobs[k].out.cpu().numpy().astype(np.float64), ref)
        assert np.array_equal(pix[k].cpu().numpy(), cnt)
    with pytest.raises(rt.Unsupported):  # one job more than a batch takes, refused before any device work
        rt.render_batch(jobs + jobs[:1], workspace=plan.ws)
    c = W.box_center(dims, sp)
    for Wd, Hd in ((32768, 2), (2, 32768)):
        hh = 40.0 * min(1.0, Hd / Wd)  # the wider side spans 80 mm
        cam = Camera(tuple(c + np.array([0.0, -120.0, 15.0])), tuple(c), (0, 0, 1), False, 0.0, hh)
        got, cnt = gpu_render(rt, torch, small["gv"], small["gtf"], cam, Wd, Hd, 0.5, 0.99)
        ref = orc.render(small["ov"], small["otf"], cam, Wd, Hd, 0.5, 0.99, tie_delta=DELTA, want_band=True)
        check(got, ref, cnt, f"{Wd}x{Hd}")
        assert (cnt > 0).mean() > 0.5


def test_one_off_batches_on_two_streams(rt, torch_mod, brain):
    """Batches of the same size issued on two streams without waiting for each
    other: each stream has its own job table, so both render what was asked."""
    torch = torch_mod
    cams = brain["cams"]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    ja = [rt.Job(brain["gv"], brain["gtf"], c, 160, 120, 0.5, 0.99) for c in cams[0:4]]
    jb = [rt.Job(brain["gv"], brain["gtf"], c, 160, 120, 0.5, 0.99) for c in cams[20:24]]
    for _ in range(3):
        rt.render_batch(ja, stream=s1)
        rt.render_batch(jb, stream=s2)
    torch.cuda.synchronize()
    for j, cam in zip(ja + jb, cams[0:4] + cams[20:24]):
        ref, _ = gpu_render(rt, torch, brain["gv"], brain["gtf"], cam, 160, 120, 0.5, 0.99)
        assert np.array_equal(j.out.cpu().numpy().astype(np.float64), ref)

# ---------------------------------------------------------------------------
# error paths that need live handles
# ---------------------------------------------------------------------------
def test_abi_errors_with_handles(rt, torch_mod, small):
    gv, gtf = small["gv"], small["gtf"]
    out = torch_mod.empty((8, 8, 4), dtype=torch_mod.float32, device="cuda")
    good = W.ortho_camera_small()
    bad = [Camera((1, 2, 3), (1, 2, 3), (0, 1, 0), True, 40.0),
           Camera((0, 0, 5), (0, 0, 0), (0, 0, 1), True, 40.0),
           Camera((0, 0, 5), (0, 0, 0), (0, 1, 0), True, 180.0),
           Camera((0, 0, 5), (0, 0, 0), (0, 1, 0), False, 0.0, 0.0),
           Camera((0, 0, float("nan")), (0, 0, 0), (0, 1, 0), True, 40.0)]
    for cam in bad:
        with pytest.raises(rt.InvalidArgument):
            rt.rt_render(gv.handle, gv.dims, None, gtf.handle, cam, 8, 8, 0.5, 0.99, None, out.data_ptr())
    for W_, H_, step, cut in [(0, 8, 0.5, 0.99), (8, 8, 0.0, 0.99), (8, 8, 0.5, 0.0), (8, 8, 0.5, 1.5),
                              (8, 8, float("inf"), 0.9)]:
        with pytest.raises(rt.InvalidArgument):
            rt.rt_render(gv.handle, gv.dims, None, gtf.handle, good, W_, H_, step, cut, None, out.data_ptr())
    with pytest.raises(rt.InvalidArgument):
        rt.rt_render(gv.handle, (64, 64, 31), None, gtf.handle, good, 8, 8, 0.5, 0.99, None, out.data_ptr())
    with pytest.raises(rt.OutOfMemory):
        buf = torch_mod.empty(100, dtype=torch_mod.uint8, device="cuda")
        src = torch_mod.zeros((4, 4, 4), dtype=torch_mod.uint8, device="cuda")
        rt.rt_create_volume(src.data_ptr(), rt.U8, (4, 4, 4), (1, 1, 1), rt.U8, rt.LAYOUT_CELLS, 0, buf.data_ptr(), 100)
    with pytest.raises(rt.InvalidArgument):
        rt.TransferFunction(np.full((16, 4), 1.5, np.float32), 0, 1)
    with pytest.raises(rt.InvalidArgument):
        rt.TransferFunction(np.zeros((16, 4), np.float32), 1, 1)
    with pytest.raises(rt.Unsupported):
        rt.rt_render(gv.handle, gv.dims, None, gtf.handle, good, 8, 8, 0.5, 0.99, None, out.data_ptr(),
                     rt.make_opts(tile=(5, 13)))


def test_volume_and_table_created_on_a_side_stream(rt, torch_mod, small):
    """Creation on a caller stream waits for the source copy made on the
    current stream; the result renders exactly like the default-stream one."""
    torch = torch_mod
    s = torch.cuda.Stream()
    gv = rt.Volume(small["np"], (1, 1, 2), storage=rt.U8, stream=s)
    gtf = rt.TransferFunction(small["tf_np"], 0, 255, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    cam = W.ortho_camera_small()
    a = rt.render(gv, gtf, cam, 96, 80, 0.5, 0.99)
    b = rt.render(small["gv"], small["gtf"], cam, 96, 80, 0.5, 0.99)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_u15_cells_bitwise_equal_u16_on_12bit_data(rt, torch_mod, brain):
    """Pairs stored as (c0, c1 - c0) interpolate with exactly the operations of
    16-bit cells: plain, batched, planned and skipping renders are bit for
    bit those of the u16 volume, sample counts included."""
    torch = torch_mod
    gv = rt.Volume(brain["np"], brain["sp"], storage=rt.U15)
    for view in (0, 11, 26):
        cam = brain["cams"][view]
        a, ca = gpu_render(rt, torch, brain["gv"], brain["gtf"], cam, 300, 220, 0.5, 0.99)
        b, cb = gpu_render(rt, torch, gv, brain["gtf"], cam, 300, 220, 0.5, 0.99)
        assert np.array_equal(a, b) and np.array_equal(ca, cb), view
    jobs16 = [rt.Job(brain["gv"], brain["gtf"], c, 160, 128, 0.5, 0.99) for c in brain["cams"][::9]]
    jobs15 = [rt.Job(gv, brain["gtf"], c, 160, 128, 0.5, 0.99, skip_empty=True) for c in brain["cams"][::9]]
    outs16 = rt.render_batch(jobs16)
    rt.BatchPlan(len(jobs15), rt.U15, skip_empty=True).launch(jobs15)
    torch.cuda.synchronize()
    for x, j in zip(outs16, jobs15):
        assert torch.equal(x, j.out)
    with pytest.raises(rt.InvalidArgument):      # a u16 plan does not take u15 volumes
        rt.BatchPlan(4, rt.U16).launch(jobs15[:1])


def test_u15_every_ray_function_bitwise_equal_u16(rt, torch_mod, brain, small):
    """Projections, thresholding (with and without skipping) and the iso-surface
    (whose shading reads six more samples per hit) give the u16 images exactly;
    an 8-bit source stored as u15 gives the images of the same values as u16."""
    torch = torch_mod
    gv = rt.Volume(brain["np"], brain["sp"], storage=rt.U15)
    cam = brain["cams"][7]
    for fn, lo, hi, sk in ((rt.MIP, 0.0, 0.0, False), (rt.XRAY, 0.0, 0.0, False),
                           (rt.AVERAGE, 0.0, 0.0, False), (rt.THRESHOLD, 1200.0, 2600.0, True),
                           (rt.ISO, 1000.0, 0.0, False)):
        a = rt.render(brain["gv"], brain["gtf"], cam, 180, 150, 0.5, 0.99, ray_function=fn, iso_value=lo,
                      iso_high=hi)
        b = rt.render(gv, brain["gtf"], cam, 180, 150, 0.5, 0.99, ray_function=fn, iso_value=lo, iso_high=hi,
                      skip_empty=sk)
        torch.cuda.synchronize()
        assert torch.equal(a, b), fn
    v8 = small["np"]
    a = rt.render(rt.Volume(v8.astype(np.uint16), (1, 1, 2), storage=rt.U16), small["gtf"], W.ortho_camera_small(),
                  96, 80, 0.5, 0.99)
    b = rt.render(rt.Volume(v8, (1, 1, 2), storage=rt.U15), small["gtf"], W.ortho_camera_small(), 96, 80, 0.5, 0.99)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_tile_orders_give_identical_images(rt, torch_mod, brain):
    """Compact and spread tile orders (and the default of each entry point)
    only change which workgroup renders a tile: images and counts are equal."""
    torch = torch_mod
    cams = brain["cams"][::7]
    for tile, wv in (((4, 16), 12), ((8, 8), 4), ((2, 32), 8)):
        for skip in (False, True):
            base = [gpu_render(rt, torch, brain["gv"], brain["gtf"], c, 200, 150, 0.5, 0.99, tile=tile,
                               waves_per_block=wv, tile_order=1, skip_empty=skip) for c in cams]
            for order in (0, 2):
                for c, (img, cnt) in zip(cams, base):
                    got = gpu_render(rt, torch, brain["gv"], brain["gtf"], c, 200, 150, 0.5, 0.99, tile=tile,
                                     waves_per_block=wv, tile_order=order, skip_empty=skip)
                    assert np.array_equal(got[0], img) and np.array_equal(got[1], cnt)
            for order in (0, 1, 2):
                outs = rt.render_batch([rt.Job(brain["gv"], brain["gtf"], c, 200, 150, 0.5, 0.99, skip_empty=skip)
                                        for c in cams], tile=tile, waves_per_block=wv, tile_order=order)
                plan = rt.BatchPlan(len(cams), rt.U16, tile=tile, waves_per_block=wv, tile_order=order,
                                    skip_empty=skip)
                pj = [rt.Job(brain["gv"], brain["gtf"], c, 200, 150, 0.5, 0.99, skip_empty=skip) for c in cams]
                plan.launch(pj)
                torch.cuda.synchronize()
                for o, j, (img, _) in zip(outs, pj, base):
                    assert np.array_equal(o.cpu().numpy().astype(np.float64), img)
                    assert np.array_equal(j.out.cpu().numpy().astype(np.float64), img)


def test_u12_brain_views_match_oracle(rt, torch_mod, orc, brain):
    """12-bit half cells hold the phantom exactly; full views against the
    oracle on the same grid, and against 16-bit storage to binary32 rounding."""
    gv = rt.Volume(brain["np"], brain["sp"], storage=rt.U12)
    for view in (2, 19):
        cam = brain["cams"][view]
        got, c = gpu_render(rt, torch_mod, gv, brain["gtf"], cam, 512, 512, 0.5, 0.99)
        ref = orc.render(brain["ov"], brain["otf"], cam, 512, 512, 0.5, 0.99, tie_delta=DELTA, want_band=True)
        check(got, ref, c, f"u12 brain view {view}")
        u16, _ = gpu_render(rt, torch_mod, brain["gv"], brain["gtf"], cam, 512, 512, 0.5, 0.99)
        assert np.abs(got - u16)[(ref.tie & 1) == 0].max() <= TOL



def test_timed_orbit_launch_matches_oracle(rt, torch_mod, orc, brain):
    """The launch the throughput figure times: all 36 orbit views in one
    graph-captured batch plan over 12-bit halves in quad bricks, 4x16-pixel
    tiles and 12 wavefronts per workgroup, in its non-counting form.  Every
    pixel of every view against the oracle (tie-aware, 1e-5) and every
    pixel's sample count (from the counting form of the same plan) exactly off
    ties; the launch-wide counter against the per-pixel counts; the
    non-counting form bitwise equal to the counting one on two replays; the
    same plan over the cell layout, and the other launch shapes the autotuner
    may pick, bitwise equal to this one."""
    torch = torch_mod
    Q = rt.LAYOUT_QUADS
    gv = rt.Volume(brain["np"], brain["sp"], storage=rt.U12, layout=Q)
    cams = brain["cams"]
    plan = rt.BatchPlan(len(cams), rt.U12, layout=Q, tile=(4, 16), waves_per_block=12)
    with pytest.raises(rt.Unsupported):  # fixed-step batches take at most 12 waves per workgroup
        rt.BatchPlan(len(cams), rt.U12, tile=(4, 16), waves_per_block=16)
    rt.BatchPlan(len(cams), rt.U12, tile=(4, 16), waves_per_block=16, skip_empty=True).close()
    pix = [torch.zeros((512, 512), dtype=torch.int32, device="cuda") for _ in cams]
    counted = [rt.Job(gv, brain["gtf"], c, 512, 512, 0.5, 0.99, pixel_counts=p) for c, p in zip(cams, pix)]
    counter = torch.zeros(1, dtype=torch.int64, device="cuda")
    plan.launch(counted, sample_counter=counter)
    torch.cuda.synchronize()
    total = int(counter.item())
    assert total == sum(int(p.to(torch.int64).sum()) for p in pix)
    timed = [rt.Job(gv, brain["gtf"], c, 512, 512, 0.5, 0.99) for c in cams]
    for _ in range(2):
        for j in timed:
            j.out.fill_(-1.0)
        plan.launch(timed)
        torch.cuda.synchronize()
        for a, b in zip(counted, timed):
            assert torch.equal(a.out, b.out)
    worst = err = 0.0
    ties = 0
    for vi, (cam, j, p) in enumerate(zip(cams, timed, pix)):
        ref = orc.render(brain["ov"], brain["otf"], cam, 512, 512, 0.5, 0.99, tie_delta=DELTA, want_band=True)
        got = j.out.cpu().numpy().astype(np.float64)
        w, e = check(got, ref, p.cpu().numpy(), f"timed orbit launch, view {vi}")
        worst, err = max(worst, w), max(err, e)
        ties += int(((ref.tie & 1) != 0).sum())
    print(f"timed orbit launch: {total} samples, 36 whole views: max err {err:.3g}, worst band distance "
          f"{worst:.3g}, {ties} tie pixels")
    gc = rt.Volume(brain["np"], brain["sp"], storage=rt.U12)
    cells = [rt.Job(gc, brain["gtf"], c, 512, 512, 0.5, 0.99) for c in cams]
    pc = rt.BatchPlan(len(cams), rt.U12, tile=(4, 16), waves_per_block=12)
    pc.launch(cells)
    torch.cuda.synchronize()
    for a, b in zip(timed, cells):
        assert torch.equal(a.out, b.out), "cell layout"
    pc.close()
    del cells, gc
    from paper_1211_5595_amd import autotune
    for (tw, th), waves in autotune.launch_candidates(skip_empty=False):
        if ((tw, th), waves) == ((4, 16), 12):
            continue
        other = [rt.Job(gv, brain["gtf"], c, 512, 512, 0.5, 0.99) for c in cams]
        p2 = rt.BatchPlan(len(cams), rt.U12, layout=Q, tile=(tw, th), waves_per_block=waves)
        p2.launch(other)
        torch.cuda.synchronize()
        for a, b in zip(timed, other):
            assert torch.equal(a.out, b.out), ((tw, th), waves)
        p2.close()


@pytest.mark.parametrize("seed", range(6))
def test_u12_random_small_cases(rt, torch_mod, orc, seed):
    """Random grids (some values above 4096, stored as 4096), tables, cameras,
    steps and cutoffs, with a plain and a batched launch."""
    rng = np.random.default_rng(1200 + seed)
    dims = tuple(int(x) for x in rng.integers(2, 60, 3))
    sp = tuple(float(x) for x in rng.uniform(0.4, 2.5, 3))
    v = rng.integers(0, 4600 if seed % 2 else 4097, size=dims[::-1], dtype=np.uint16)
    v = ((v.astype(np.int64) + np.roll(v, 1, 0) + np.roll(v, 1, 1)) // 3).astype(np.uint16)
    t = W.random_tf(int(rng.integers(64, 4097)), seed + 120, alpha_max=float(rng.uniform(0.05, 0.9)))
    cam = W.random_camera(rng, dims, sp)
    Wd, Hd = int(rng.integers(1, 120)), int(rng.integers(1, 100))
    step, cutoff = float(rng.uniform(0.2, 1.2)), float(rng.uniform(0.6, 1.0))
    gv, gtf = rt.Volume(v, sp, storage=rt.U12), rt.TransferFunction(t, 0, 4600)
    got, c = gpu_render(rt, torch_mod, gv, gtf, cam, Wd, Hd, step, cutoff)
    ref = orc.render(orc.Volume(np.minimum(v, 4096), sp), orc.TF(t, 0, 4600), cam, Wd, Hd, step, cutoff,
                     tie_delta=DELTA, want_band=True)
    check(got, ref, c, f"u12 seed {seed} dims {dims}")
    out = rt.render_batch([rt.Job(gv, gtf, cam, Wd, Hd, step, cutoff)])[0]
    torch_mod.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().astype(np.float64), got)


def test_u12_from_u8_source(rt, torch_mod, orc, small):
    gv = rt.Volume(small["np"], (1, 1, 2), storage=rt.U12)
    got, c = gpu_render(rt, torch_mod, gv, small["gtf"], W.ortho_camera_small(), 128, 128, 0.5, 0.99)
    ref = orc.render(small["ov"], small["otf"], W.ortho_camera_small(), 128, 128, 0.5, 0.99, tie_delta=DELTA,
                     want_band=True)
    check(got, ref, c, "u12 from u8")
    with pytest.raises(rt.InvalidArgument):     # binary32 source: not integer data
        rt.Volume(small["np"].astype(np.float32), (1, 1, 2), storage=rt.U12)


def test_u15_clamps_above_32767(rt, torch_mod, orc):
    """Values above 32767 are stored as 32767; the render equals the oracle on
    the clamped field."""
    rng = np.random.default_rng(15)
    dims, sp = (29, 23, 17), (0.8, 1.0, 1.3)
    v = rng.integers(0, 65536, size=dims[::-1], dtype=np.uint16)
    v = ((v.astype(np.int64) + np.roll(v, 1, 0) + np.roll(v, 1, 2)) // 3).astype(np.uint16)
    t = W.random_tf(1024, 61, alpha_max=0.3)
    cam = W.random_camera(rng, dims, sp)
    gv = rt.Volume(v, sp, storage=rt.U15)
    got, c = gpu_render(rt, torch_mod, gv, rt.TransferFunction(t, 0, 40000), cam, 70, 50, 0.5, 0.99)
    ref = orc.render(orc.Volume(np.minimum(v, 32767), sp), orc.TF(t, 0, 40000), cam, 70, 50, 0.5, 0.99,
                     tie_delta=DELTA, want_band=True)
    check(got, ref, c, "u15 clamped")
    assert (v > 32767).any()


@pytest.mark.parametrize("step,unit", [(0.5, 0.9), (0.25, 0.9), (0.8, 0.3)])
def test_opacity_correction_matches_oracle(rt, torch_mod, orc, brain, step, unit):
    """Opacity correction to a unit distance (table entries corrected when
    staged): full brain view against the oracle, for u16 and u12 storage, with
    and without skipping (bitwise equal), plain and batched (bitwise equal)."""
    torch = torch_mod
    cam = brain["cams"][9]
    ref = orc.render(brain["ov"], brain["otf"], cam, 256, 256, step, 0.99, tie_delta=DELTA, want_band=True,
                     opacity_unit=unit)
    gv12 = rt.Volume(brain["np"], brain["sp"], storage=rt.U12)
    for gv in (brain["gv"], gv12):
        got, c = gpu_render(rt, torch, gv, brain["gtf"], cam, 256, 256, step, 0.99, opacity_unit_distance=unit)
        check(got, ref, c, f"opacity unit {unit} step {step}")
        sk, cs = gpu_render(rt, torch, gv, brain["gtf"], cam, 256, 256, step, 0.99, opacity_unit_distance=unit,
                            skip_empty=True)
        assert np.array_equal(sk, got) and np.array_equal(cs, c)
        jobs = [rt.Job(gv, brain["gtf"], cam, 256, 256, step, 0.99, opacity_unit_distance=unit),
                rt.Job(gv, brain["gtf"], cam, 256, 256, step, 0.99),               # same table, no correction
                rt.Job(gv, brain["gtf"], cam, 256, 256, step, 0.99, opacity_unit_distance=unit, skip_empty=True)]
        outs = rt.render_batch(jobs)
        plain = rt.render(gv, brain["gtf"], cam, 256, 256, step, 0.99)
        torch.cuda.synchronize()
        assert np.array_equal(outs[0].cpu().numpy().astype(np.float64), got)
        assert np.array_equal(outs[2].cpu().numpy().astype(np.float64), got)
        assert torch.equal(outs[1], plain)


def test_opacity_correction_thresholding_and_slab(rt, torch_mod, orc, small):
    torch = torch_mod
    cam = W.ortho_camera_small()
    for fn, lo, hi in ((rt.THRESHOLD, 100.0, 230.0), (rt.COMPOSITE, 0.0, 0.0)):
        got, c = gpu_render(rt, torch, small["gv"], small["gtf"], cam, 128, 128, 0.45, 0.99,
                            opacity_unit_distance=1.7, ray_function=fn, iso_value=lo, iso_high=hi)
        ref = orc.render(small["ov"], small["otf"], cam, 128, 128, 0.45, 0.99, tie_delta=DELTA, want_band=True,
                         opacity_unit=1.7, ray_function=fn, iso_value=lo, iso_high=hi)
        keep = (ref.tie & 8) == 0
        dist = np.maximum(np.maximum(ref.band_lo - got, got - ref.band_hi), 0.0).max(-1)
        assert dist[keep].max() <= TOL
    # a uniform slab's opacity depends on its thickness only: 1-(1-a)^(L/u) at every step
    v = np.full((4, 4, 4), 7, dtype=np.uint8)
    t = np.zeros((8, 4), np.float32)
    t[:, :3], t[:, 3] = 0.5, 0.1
    gv, gtf = rt.Volume(v, (1, 1, 1), storage=rt.U8), rt.TransferFunction(t, 0, 10)
    slab = W.Camera((1.5, 1.5, -10.0), (1.5, 1.5, 0.0), (0, 1, 0), False, 0.0, 1.0)
    A = 1 - (1 - float(np.float32(0.1))) ** (3.0 / 1.5)
    for step in (0.3, 0.5, 0.7, 1.1):
        img, _ = gpu_render(rt, torch, gv, gtf, slab, 2, 2, step, 1.0, opacity_unit_distance=1.5)
        np.testing.assert_allclose(img[..., 3], A, atol=2e-6)
    with pytest.raises(rt.InvalidArgument):
        rt.render(gv, gtf, slab, 2, 2, 0.5, 1.0, opacity_unit_distance=-1.0)


@pytest.mark.parametrize("storage", ["U16", "U12", "U8_BRICKSCALED"])
def test_extreme_steps_tables_and_cutoffs(rt, torch_mod, orc, storage):
    """Steps from 0.05 voxel (rays of thousands of samples) to 6 voxels (rays of
    one or two, shorter than the single-view kernel's ring of in-flight cells),
    the smallest and largest tables, a cutoff reached at the first sample, a
    value window narrower than the data, and one-pixel-wide images; plain and
    batched renders equal the oracle, and each other bit for bit."""
    torch = torch_mod
    dims, sp = (40, 33, 21), (1.0, 0.8, 1.6)
    v = W.phantom_brain(77, dims=dims, spacing=sp)
    if storage == "U8_BRICKSCALED":
        gv, ov = rt.Volume(v, sp, storage=rt.U8_BRICKSCALED, brick=8), orc.Volume.from_u8_bricks(v, sp, 8)
    else:
        gv, ov = rt.Volume(v, sp, storage=getattr(rt, storage)), orc.Volume(v, sp)
    rng = np.random.default_rng(91)
    cases = [(0.05, W.random_tf(4096, 1, alpha_max=0.02), 0.0, 4095.0, 0.99, 24, 20),
             (6.0, W.random_tf(2, 2, alpha_max=0.9), 0.0, 4095.0, 1.0, 31, 17),
             (3.3, W.random_tf(256, 3, alpha_max=0.5), 500.0, 1500.0, 0.99, 1, 40),
             (0.7, W.random_tf(64, 4, alpha_max=1.0), 0.0, 4095.0, 0.01, 40, 1),
             (1.9, W.random_tf(4096, 5, alpha_max=0.3), 0.0, 4095.0, 0.5, 33, 29)]
    for step, table, lo, hi, cutoff, Wd, Hd in cases:
        cam = W.random_camera(rng, dims, sp)
        gtf = rt.TransferFunction(table, lo, hi)
        got, c = gpu_render(rt, torch, gv, gtf, cam, Wd, Hd, step, cutoff)
        ref = orc.render(ov, orc.TF(table, lo, hi), cam, Wd, Hd, step, cutoff, tie_delta=DELTA, want_band=True)
        check(got, ref, c, f"{storage} step {step} K {table.shape[0]} cutoff {cutoff} {Wd}x{Hd}")
        skip, cs = gpu_render(rt, torch, gv, gtf, cam, Wd, Hd, step, cutoff, skip_empty=True)
        assert np.array_equal(skip, got) and np.array_equal(cs, c)
        out = rt.render_batch([rt.Job(gv, gtf, cam, Wd, Hd, step, cutoff)])[0]
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().astype(np.float64), got)
