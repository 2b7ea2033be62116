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
    assert res["ms"] <= res["timings_ms"][str(((8, 8), 16))] + 1e-9
    assert at.tune_launch(vol, tf, cams, 384, 384, cache=cache) == res            # served from the cache
    a = rt.render(vol, tf, cams[2], 384, 384)
    b = rt.render(vol, tf, cams[2], 384, 384, tile=tuple(res["tile"]), waves_per_block=res["waves_per_block"])
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    lay = at.tune_layout(W.phantom_brain(9, dims=(64, 64, 48), spacing=sp), sp, rt.U16, tf, cams[:2], 128, 128,
                         reps=1)
    assert lay["layout"] in (rt.LAYOUT_CELLS, rt.LAYOUT_POLY, rt.LAYOUT_LINEAR)
