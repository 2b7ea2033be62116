"""The two forms of a batch plan: the persistent form (workgroups pull
blocks from a queue) and the latency form for small batches (one workgroup
per block, sized to the batch).  Both render each view exactly as rt_render
does (arXiv:1211.5595, Sections 3.2 and 4.1-4.2: only the launch differs),
so images, per-pixel sample counts and the launch-wide sample count must be
bitwise equal between the forms, for every ray function, with and without
empty-space skipping, in both storage layouts of 12-bit data."""
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
def scene(rt):
    sp = (0.9, 0.9, 1.2)
    dims = [(128, 128, 64), (192, 192, 96), (256, 256, 160)]
    grids = [W.phantom_brain(500 + i, dims=d, spacing=sp) for i, d in enumerate(dims)]
    tfs = [rt.TransferFunction(W.random_tf(4096, 510 + i, alpha_max=0.05), 0.0, 4095.0) for i in range(4)]
    rng = np.random.default_rng(520)
    cams = [(i % 3, W.random_camera(rng, dims[i % 3], sp)) for i in range(12)]
    return dict(sp=sp, dims=dims, grids=grids, tfs=tfs, cams=cams)


def _jobs(rt, vols, scene, sides, fns, skip, counts):
    import torch
    out = []
    for k, ((vi, cam), s) in enumerate(zip(scene["cams"], sides)):
        fn, lo, hi = fns[k % len(fns)]
        c = torch.zeros((s[1], s[0]), dtype=torch.int32, device="cuda") if counts else None
        out.append(rt.Job(vols[vi], scene["tfs"][k % 4], cam, s[0], s[1], 0.5 + 0.25 * (k % 3), 0.99 - 0.1 * (k % 2),
                          pixel_counts=c, ray_function=fn, iso_value=lo, iso_high=hi, skip_empty=skip))
    return out


# ragged sizes: tails in both directions, a one-pixel view, a tall strip.  12
# views take the latency form's workspace kernel, 2..6 its kernel-argument
# kernel, one view the single-view kernel.
SIDES = [(257, 131), (64, 64), (1, 1), (320, 200), (33, 700), (128, 96), (512, 384), (77, 77), (256, 256),
         (19, 300), (200, 19), (640, 480)]


@pytest.mark.parametrize("n", [12, 5, 2, 1])
@pytest.mark.parametrize("layout", ["QUADS", "CELLS"])
@pytest.mark.parametrize("skip", [False, True])
def test_forms_bitwise_equal(rt, scene, layout, skip, n):
    import torch
    L = getattr(rt, "LAYOUT_" + layout)
    vols = [rt.Volume(g, scene["sp"], storage=rt.U12, layout=L) for g in scene["grids"]]
    fns = [(rt.COMPOSITE, 0.0, 0.0), (rt.COMPOSITE, 0.0, 0.0), (rt.MIP, 0.0, 0.0), (rt.THRESHOLD, 1200.0, 2600.0),
           (rt.ISO, 1000.0, 0.0), (rt.AVERAGE, 0.0, 0.0)]
    sides = SIDES[:n] if n != 1 else [SIDES[3]]
    res = {}
    for form in (1, 2):
        plan = rt.BatchPlan(len(sides), rt.U12, layout=L, skip_empty=skip, tile_order=2, batch_form=form)
        jobs = _jobs(rt, vols, scene, sides, fns, skip, counts=True)
        counter = torch.zeros(1, dtype=torch.int64, device="cuda")
        plan.launch(jobs, sample_counter=counter)
        torch.cuda.synchronize()
        assert int(counter.item()) == sum(int(j.pixel_counts.to(torch.int64).sum()) for j in jobs)
        res[form] = (jobs, int(counter.item()))
        plan.close()
    (ja, ca), (jb, cb) = res[1], res[2]
    assert ca == cb
    for a, b in zip(ja, jb):
        assert torch.equal(a.out, b.out) and torch.equal(a.pixel_counts, b.pixel_counts)
    # and each view as rt_render gives it alone
    for j in jb[:6]:
        img = rt.render(j.volume, j.tf, j.camera, j.width, j.height, j.step_vox, j.alpha_cutoff,
                        ray_function=j.ray_function, iso_value=j.iso_value, iso_high=j.iso_high, skip_empty=skip)
        torch.cuda.synchronize()
        assert torch.equal(img, j.out)


def test_automatic_form_by_size(rt, scene):
    """batch_form 0: batches up to rt_batch_latency_pixels() take the latency
    form, larger ones the persistent form; the same images either way, on
    consecutive launches of one plan that switch between the forms."""
    import torch
    lim = rt.rt_batch_latency_pixels()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert lim == cus * 4 * 4 * 64
    vols = [rt.Volume(g, scene["sp"], storage=rt.U12, layout=rt.LAYOUT_QUADS) for g in scene["grids"]]
    auto = rt.BatchPlan(12, rt.U12, layout=rt.LAYOUT_QUADS, skip_empty=True)
    ref = rt.BatchPlan(12, rt.U12, layout=rt.LAYOUT_QUADS, skip_empty=True, batch_form=1)
    fns = [(rt.COMPOSITE, 0.0, 0.0)]
    for sides in ([(256, 256)], [(512, 512)], [(512, 512), (64, 64)], [(1024, 1024)] * 3, [(300, 200)] * 12):
        a = _jobs(rt, vols, scene, sides, fns, True, counts=False)
        b = _jobs(rt, vols, scene, sides, fns, True, counts=False)
        auto.launch(a)
        ref.launch(b)
        torch.cuda.synchronize()
        for x, y in zip(a, b):
            assert torch.equal(x.out, y.out), sides


def test_batch_form_argument_checked(rt):
    with pytest.raises(rt.InvalidArgument):
        rt.BatchPlan(4, rt.U12, batch_form=3)
    with pytest.raises(rt.InvalidArgument):
        rt.BatchPlan(4, rt.U12, batch_form=-1)


def test_table_update_changes_size_in_place(rt, scene):
    """A table handle created with 4096 entries takes smaller tables in place
    (as the server's slots do); renders equal those of a fresh handle; a table
    larger than the handle's buffers is refused."""
    import torch
    vol = rt.Volume(scene["grids"][1], scene["sp"], storage=rt.U12, layout=rt.LAYOUT_QUADS)
    vi, cam = scene["cams"][1]
    big = W.random_tf(4096, 61, alpha_max=0.05)
    tf = rt.TransferFunction(big, 0.0, 4095.0)
    for K, seed in ((200, 62), (2, 63), (4096, 64), (37, 65)):
        t = W.random_tf(K, seed, alpha_max=0.3)
        tf.update(t)
        a = rt.render(vol, tf, cam, 96, 80, skip_empty=True)
        fresh = rt.TransferFunction(t, 0.0, 4095.0)
        b = rt.render(vol, fresh, cam, 96, 80, skip_empty=True)
        torch.cuda.synchronize()
        assert torch.equal(a, b), K
    small = rt.TransferFunction(W.random_tf(64, 66), 0.0, 4095.0)
    with pytest.raises(rt.OutOfMemory):
        small.update(big)


def test_table_updates_back_to_back_keep_each_render(rt, scene):
    """A table handle updated again and again with a render after each
    update, with no synchronisation in between: every render sees the table
    given just before it (the upload kernel reads the handle's staging buffer
    on the stream, and an update waits for the previous upload before
    rewriting that buffer)."""
    import torch
    vol = rt.Volume(scene["grids"][0], scene["sp"], storage=rt.U12, layout=rt.LAYOUT_QUADS)
    vi, cam = scene["cams"][0]
    tables = [W.random_tf(K, 80 + i, alpha_max=0.3) for i, K in enumerate((4096, 300, 4096, 17, 2048, 4096, 5, 1000))]
    tf = rt.TransferFunction(tables[0], 0.0, 4095.0)
    got = []
    for t in tables:
        tf.update(t)
        got.append(rt.render(vol, tf, cam, 72, 64, skip_empty=True))
    torch.cuda.synchronize()
    for k, t in enumerate(tables):
        fresh = rt.TransferFunction(t, 0.0, 4095.0)
        ref = rt.render(vol, fresh, cam, 72, 64, skip_empty=True)
        torch.cuda.synchronize()
        assert torch.equal(got[k], ref), k
