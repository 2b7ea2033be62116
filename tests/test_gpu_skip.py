"""Empty-space skipping on the GPU (through the C ABI).

Skipping only steps over samples whose table opacity is exactly zero, which
leave colour and transmittance unchanged bit for bit, so every image and every
per-pixel sample count must be identical with and without it, for every
storage type and layout, in plain and batched launches.  The per-brick value
ranges it relies on are checked against the grid itself, and one view against
the FP64 oracle.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


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


def render_pair(rt, torch, vol, tf, cam, W_, H_, step=0.5, cutoff=0.99, **kw):
    out = []
    for skip in (False, True):
        counts = torch.zeros((H_, W_), dtype=torch.int32, device="cuda")
        img = rt.render(vol, tf, cam, W_, H_, step, cutoff, pixel_counts=counts, skip_empty=skip, **kw)
        torch.cuda.synchronize()
        out.append((img.cpu().numpy(), counts.cpu().numpy()))
    return out


def assert_identical(pair, what):
    (a, ca), (b, cb) = pair
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), f"{what}: images differ"
    assert np.array_equal(ca, cb), f"{what}: sample counts differ"


@pytest.fixture(scope="module")
def brain(rt):
    dims, sp = (256, 256, 160), (0.9, 0.9, 1.2)
    v = W.phantom_brain(11)
    return dict(np=v, dims=dims, sp=sp, gv=rt.Volume(v, sp, storage=rt.U16),
                tf=rt.TransferFunction(W.random_tf(4096, 12, alpha_max=0.05), 0, 4095),
                cams=W.orbit_cameras(dims, sp, 36))


@pytest.mark.parametrize("view", [0, 7, 13, 22, 30])
def test_brain_views_identical(rt, torch_mod, brain, view):
    pair = render_pair(rt, torch_mod, brain["gv"], brain["tf"], brain["cams"][view], 512, 512)
    assert_identical(pair, f"view {view}")


def test_brain_view_matches_oracle(rt, torch_mod, orc, brain):
    from test_gpu_parity import check
    cam = brain["cams"][4]
    (_, _), (img, c) = render_pair(rt, torch_mod, brain["gv"], brain["tf"], cam, 256, 256)
    ref = orc.render(orc.Volume(brain["np"], brain["sp"]), orc.TF(W.random_tf(4096, 12, alpha_max=0.05), 0, 4095),
                     cam, 256, 256, 0.5, 0.99, tie_delta=1e-6, want_band=True)
    check(img.astype(np.float64), ref, c, "skip brain view 4")


@pytest.mark.parametrize("storage,layout,brick", [
    ("U8", "LAYOUT_CELLS", 0), ("U8", "LAYOUT_LINEAR", 0), ("U8", "LAYOUT_POLY", 0),
    ("U16", "LAYOUT_LINEAR", 0), ("U16", "LAYOUT_POLY", 0),
    ("F16", "LAYOUT_CELLS", 0), ("F16", "LAYOUT_LINEAR", 0),
    ("F32", "LAYOUT_CELLS", 0), ("F32", "LAYOUT_LINEAR", 0),
    ("U8_BRICKSCALED", "LAYOUT_CELLS", 16), ("U8_BRICKSCALED", "LAYOUT_BRICKS", 8),
    ("U15", "LAYOUT_CELLS", 0), ("U12", "LAYOUT_CELLS", 0),
])
def test_storage_and_layouts_identical(rt, torch_mod, brain, storage, layout, brick):
    v = brain["np"]
    vmax = 4095
    if storage == "U8":
        v = (v >> 4).astype(np.uint8)
        vmax = 255
    gv = rt.Volume(v, brain["sp"], storage=getattr(rt, storage), layout=getattr(rt, layout), brick=brick)
    tf = rt.TransferFunction(W.random_tf(1024, 31, alpha_max=0.1), 0, vmax)
    for view in (3, 19):
        pair = render_pair(rt, torch_mod, gv, tf, brain["cams"][view], 200, 150)
        assert_identical(pair, f"{storage}/{layout} view {view}")


@pytest.mark.parametrize("seed", range(10))
def test_random_volumes_identical(rt, torch_mod, seed):
    """Random grids with a random air fraction, random tables (some with wide
    zero-opacity ranges), random cameras, steps and cutoffs."""
    rng = np.random.default_rng(500 + seed)
    dims = tuple(int(x) for x in rng.integers(2, 90, 3))
    sp = tuple(float(x) for x in rng.uniform(0.4, 2.5, 3))
    v = rng.integers(0, 4096, size=dims[::-1], dtype=np.uint16)
    air = rng.uniform(0.2, 0.9)
    v[rng.uniform(size=v.shape) < air] = 0
    v = np.ascontiguousarray(np.minimum(v, np.roll(v, 1, axis=int(seed % 3))))    # spatially coherent air
    t = W.random_tf(int(rng.integers(16, 4097)), seed + 90, alpha_max=float(rng.uniform(0.05, 1.0)),
                    air_cut=float(rng.uniform(0.0, 0.5)))
    gv = rt.Volume(v, sp, storage=rt.U16)
    tf = rt.TransferFunction(t, 0, 4095)
    cam = W.random_camera(rng, dims, sp)
    pair = render_pair(rt, torch_mod, gv, tf, cam, int(rng.integers(1, 160)), int(rng.integers(1, 120)),
                       step=float(rng.uniform(0.1, 1.5)), cutoff=float(rng.uniform(0.5, 1.0)))
    assert_identical(pair, f"seed {seed} dims {dims}")


def test_all_transparent_and_all_opaque_tables(rt, torch_mod, brain):
    cam = brain["cams"][9]
    clear = np.zeros((64, 4), np.float32)
    (a, ca), (b, cb) = render_pair(rt, torch_mod, brain["gv"], rt.TransferFunction(clear, 0, 4095), cam, 128, 128,
                                   bg=(0.1, 0.2, 0.3, 0.4))
    assert np.array_equal(a, b) and np.array_equal(ca, cb)
    assert np.array_equal(b, np.broadcast_to(np.float32([0.1, 0.2, 0.3, 0.4]), b.shape))
    dense = np.full((64, 4), 0.01, np.float32)
    pair = render_pair(rt, torch_mod, brain["gv"], rt.TransferFunction(dense, 0, 4095), cam, 128, 128)
    assert_identical(pair, "no empty brick")


def test_skip_ranges_bound_the_grid(rt, torch_mod):
    """For integer data the stored range of a skip brick is exactly the min
    and max over the padded nodes its cells touch."""
    dims = (37, 21, 18)
    rng = np.random.default_rng(3)
    v = rng.integers(0, 4096, size=dims[::-1], dtype=np.uint16)
    gv = rt.Volume(v, (1, 1, 1), storage=rt.U16)
    torch_mod.cuda.synchronize()
    nb = [(n + 1 + 7) // 8 for n in dims]
    ns = [(b + 3) // 4 for b in nb]
    r256 = lambda x: (x + 255) // 256 * 256
    total = gv.nbytes
    start = total - r256(ns[0] * ns[1] * ns[2] * 8) - r256(nb[0] * nb[1] * nb[2] * 8)
    raw = gv.buf.cpu().numpy()[start: total]
    rng_ = raw[: nb[0] * nb[1] * nb[2] * 8].view(np.float32).reshape(nb[2], nb[1], nb[0], 2)
    sup = raw[r256(nb[0] * nb[1] * nb[2] * 8):][: ns[0] * ns[1] * ns[2] * 8].view(np.float32).reshape(
        ns[2], ns[1], ns[0], 2)
    g = np.pad(v.astype(np.float64), 1, mode="edge")            # padded nodes 0..n+1
    for bz in range(nb[2]):
        for by in range(nb[1]):
            for bx in range(nb[0]):
                blk = g[8 * bz: 8 * bz + 9, 8 * by: 8 * by + 9, 8 * bx: 8 * bx + 9]
                assert rng_[bz, by, bx, 0] == blk.min() and rng_[bz, by, bx, 1] == blk.max()
    for qz in range(ns[2]):
        for qy in range(ns[1]):
            for qx in range(ns[0]):
                blk = g[32 * qz: 32 * qz + 33, 32 * qy: 32 * qy + 33, 32 * qx: 32 * qx + 33]
                assert sup[qz, qy, qx, 0] == blk.min() and sup[qz, qy, qx, 1] == blk.max()


def test_batches_and_plans_identical(rt, torch_mod, brain):
    """Jobs with and without skipping, compositing and a projection, in one
    persistent launch and in a skipping plan: bit for bit the plain images."""
    torch = torch_mod
    tf_p = rt.TransferFunction(W.random_tf(4096, 12, alpha_max=0.6), 0, 4095)
    specs = []
    for k in range(8):
        fn = rt.MIP if k == 5 else rt.COMPOSITE
        specs.append((fn, brain["tf"] if fn == rt.COMPOSITE else tf_p, brain["cams"][4 * k + 2], 96 + 32 * k,
                      90 + 10 * k, k % 2 == 0))
    plain = [rt.render(brain["gv"], tf, cam, Wd, Hd, 0.5, 0.99, ray_function=fn)
             for fn, tf, cam, Wd, Hd, _ in specs]
    jobs = [rt.Job(brain["gv"], tf, cam, Wd, Hd, 0.5, 0.99, ray_function=fn, skip_empty=sk)
            for fn, tf, cam, Wd, Hd, sk in specs]
    outs = rt.render_batch(jobs)
    plan = rt.BatchPlan(len(jobs), rt.U16, skip_empty=True)
    jobs2 = [rt.Job(brain["gv"], tf, cam, Wd, Hd, 0.5, 0.99, ray_function=fn, skip_empty=sk)
             for fn, tf, cam, Wd, Hd, sk in specs]
    c_plan = torch.zeros(1, dtype=torch.int64, device="cuda")
    plan.launch(jobs2, sample_counter=c_plan)
    c_plain = torch.zeros(1, dtype=torch.int64, device="cuda")
    rt.render_batch([rt.Job(brain["gv"], tf, cam, Wd, Hd, 0.5, 0.99, ray_function=fn)
                     for fn, tf, cam, Wd, Hd, _ in specs], sample_counter=c_plain)
    torch.cuda.synchronize()
    for a, b, j in zip(plain, outs, jobs2):
        assert torch.equal(a, b) and torch.equal(a, j.out)
    assert int(c_plan.item()) == int(c_plain.item())
