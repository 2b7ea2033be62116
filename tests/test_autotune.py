"""Autotuner: cache keys and persistence on the CPU; on the GPU, the tuned
launch renders the same image bit for bit and is no slower than the default."""
import numpy as np
import pytest

from paper_1211_5595_amd import autotune as at


def test_size_classes_and_keys():
    assert at.size_class(1) == 0 and at.size_class(1023) == 9 and at.size_class(1024) == 10
    k1 = at.launch_key("gfx950", 1, 0, (256, 256, 160), 512, 512)
    k2 = at.launch_key("gfx950", 1, 0, (250, 256, 160), 600, 512)     # same buckets
    k3 = at.launch_key("gfx950", 1, 0, (512, 512, 256), 512, 512)
    assert k1 == k2 and k1 != k3


def test_pick_best_and_cache_roundtrip(tmp_path):
    best, table = at.pick_best([(8, 8), (16, 4), (4, 16)], lambda c: {(8, 8): 3.0, (16, 4): 2.5, (4, 16): 4.0}[c])
    assert best == (16, 4) and table[str((16, 4))] == 2.5
    path = str(tmp_path / "sub" / "cache.json")
    c = at.Cache(path)
    c.put("k", {"tile": [16, 4], "waves_per_block": 8})
    assert at.Cache(path).get("k") == {"tile": [16, 4], "waves_per_block": 8}
    assert at.Cache(str(tmp_path / "missing.json")).get("k") is None


@pytest.mark.gpu
def test_tuned_launch_is_bitwise_equal_and_not_slower(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1211_5595_amd as rt
    import workloads as W
    dims, sp = (160, 160, 96), (0.9, 0.9, 1.2)
    vol = rt.Volume(W.phantom_brain(9, dims=dims, spacing=sp), sp, storage=rt.U16)
    tf = rt.TransferFunction(W.random_tf(4096, 4, alpha_max=0.05), 0, 4095)
    cams = W.orbit_cameras(dims, sp, 6)
    cache = at.Cache(str(tmp_path / "c.json"))
    res = at.tune_launch(vol, tf, cams, 384, 384, cache=cache, reps=2)
    assert tuple(res["tile"]) in at.TILES and res["waves_per_block"] in at.WAVES
    assert res["ms"] <= res["timings_ms"][str(((8, 8), 12))] + 1e-9
    assert at.tune_launch(vol, tf, cams, 384, 384, cache=cache) == res            # served from the cache
    a = rt.render(vol, tf, cams[2], 384, 384)
    b = rt.render(vol, tf, cams[2], 384, 384, tile=tuple(res["tile"]), waves_per_block=res["waves_per_block"])
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    lay = at.tune_layout(W.phantom_brain(9, dims=(64, 64, 48), spacing=sp), sp, rt.U16, tf, cams[:2], 128, 128,
                         reps=1)
    assert lay["layout"] in (rt.LAYOUT_CELLS, rt.LAYOUT_POLY, rt.LAYOUT_LINEAR, rt.LAYOUT_QUADS)


def test_exact_storage_candidates():
    """Only encodings that hold the grid exactly are offered."""
    import paper_1211_5595_amd as rt
    u12 = np.array([[[0, 4096]]], dtype=np.uint16)
    u15 = np.array([[[0, 4097]]], dtype=np.uint16)
    u16 = np.array([[[0, 32768]]], dtype=np.uint16)
    c12, c15, c16 = at.exact_storages(u12), at.exact_storages(u15), at.exact_storages(u16)
    assert (rt.U12, rt.LAYOUT_CELLS) in c12 and (rt.U15, rt.LAYOUT_CELLS) in c12
    assert (rt.U12, rt.LAYOUT_CELLS) not in c15 and (rt.U15, rt.LAYOUT_CELLS) in c15
    assert all(s == rt.U16 for s, _ in c16)
    c8 = at.exact_storages(np.array([[[0, 255]]], dtype=np.uint8))
    assert (rt.U8, rt.LAYOUT_CELLS) in c8 and (rt.U12, rt.LAYOUT_CELLS) in c8
    assert at.exact_storages(np.zeros((2, 2, 2), np.float32)) == []


@pytest.mark.gpu
def test_tuned_storage_renders_the_same_grid(tmp_path, orc):
    """Every storage the tuner may pick holds the same grid: the chosen one
    (and every other candidate) renders the oracle's image of the uint16 grid
    to the binary32 bar, 1e-5 inside the oracle's early-termination tie band,
    with sample counts equal off ties."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1211_5595_amd as rt
    import workloads as W
    dims, sp = (128, 112, 80), (0.9, 0.9, 1.2)
    v = W.phantom_brain(21, dims=dims, spacing=sp)
    table = W.random_tf(4096, 6, alpha_max=0.05)
    tf = rt.TransferFunction(table, 0, 4095)
    cams = W.orbit_cameras(dims, sp, 4)
    res = at.tune_storage(v, sp, tf, cams, 256, 256, reps=1, cache=at.Cache(str(tmp_path / "s.json")))
    assert (res["storage"], res["layout"]) in at.exact_storages(v)
    assert len(res["timings_ms"]) == len(at.exact_storages(v))
    ref = orc.render(orc.Volume(v, sp), orc.TF(table, 0, 4095), cams[1], 256, 256, 0.5, 0.99, tie_delta=1e-6,
                     want_band=True)
    ties = (ref.tie & 7) != 0
    for storage, layout in at.exact_storages(v):
        counts = torch.zeros((256, 256), dtype=torch.int32, device="cuda")
        img = rt.render(rt.Volume(v, sp, storage=storage, layout=layout), tf, cams[1], 256, 256, pixel_counts=counts)
        torch.cuda.synchronize()
        got = img.cpu().numpy().astype(np.float64)
        dist = np.maximum(np.maximum(ref.band_lo - got, got - ref.band_hi), 0.0)
        assert dist.max() <= 1e-5, (storage, layout, float(dist.max()))
        assert np.abs(got - ref.image)[~((ref.tie & 1) != 0)].max() <= 1e-5, (storage, layout)
        assert (counts.cpu().numpy() == ref.counts)[~ties].all(), (storage, layout)


@pytest.mark.gpu
def test_tune_batch_picks_a_candidate_and_renders_the_same(tmp_path):
    """The whole-batch tuner times every (tile, waves) candidate on the batch
    itself and picks the fastest; the tuned plan's images equal the default
    plan's bit for bit (the shape never changes a pixel)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1211_5595_amd as rt
    import workloads as W
    sp = (0.9, 0.9, 1.2)
    vols = [rt.Volume(W.phantom_brain(40 + i, dims=d, spacing=sp), sp, storage=rt.U12, layout=rt.LAYOUT_QUADS)
            for i, d in enumerate([(96, 96, 48), (128, 128, 64)])]
    tf = rt.TransferFunction(W.random_tf(4096, 41, alpha_max=0.05), 0, 4095)
    rng = np.random.default_rng(42)
    views = [(i % 2, W.random_camera(rng, vols[i % 2].dims, sp), 64 * (2 + i % 3)) for i in range(6)]
    jobs = [rt.Job(vols[v], tf, c, s, s, 0.5, 0.99) for v, c, s in views]
    cache = at.Cache(str(tmp_path / "b.json"))
    res = at.tune_batch(jobs, rt.U12, rt.LAYOUT_QUADS, reps=1, cache=cache)
    assert len(res["timings_ms"]) == len(at.launch_candidates(False))
    assert res["ms"] == min(res["timings_ms"].values())
    assert at.tune_batch(jobs, rt.U12, rt.LAYOUT_QUADS, cache=cache) == res      # served from the cache
    tuned = rt.BatchPlan(6, rt.U12, layout=rt.LAYOUT_QUADS, tile=tuple(res["tile"]),
                         waves_per_block=res["waves_per_block"], batch_form=1)
    ref = [rt.Job(vols[v], tf, c, s, s, 0.5, 0.99) for v, c, s in views]
    tuned.launch(jobs)
    rt.BatchPlan(6, rt.U12, layout=rt.LAYOUT_QUADS, batch_form=1).launch(ref)
    torch.cuda.synchronize()
    for a, b in zip(jobs, ref):
        assert torch.equal(a.out, b.out)
