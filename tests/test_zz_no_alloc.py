"""rt_render_batch_noalloc (workspace in the library's own device array)
against rt_render_batch (caller's workspace), through the C ABI: bitwise
equal images, per-pixel sample counts and launch-wide counters on two calls
in a row, the second with fewer and smaller views (the array keeps the first
call's contents), and the job limit refused before any device work."""
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


def _jobs(rt, torch, vol, tf, cams, side, skip=False):
    out = []
    for c in cams:
        j = rt.Job(vol, tf, c, side, side, 0.5, 0.99, skip_empty=skip,
                   pixel_counts=torch.zeros((side, side), dtype=torch.int32, device="cuda"))
        j.out.fill_(-1.0)
        out.append(j)
    return out


def _run_pair(rt, torch, vol, tf, cams, side, skip=False):
    ref = _jobs(rt, torch, vol, tf, cams, side, skip)
    got = _jobs(rt, torch, vol, tf, cams, side, skip)
    c_ref = torch.zeros(1, dtype=torch.int64, device="cuda")
    c_got = torch.zeros(1, dtype=torch.int64, device="cuda")
    rt.render_batch(ref, sample_counter=c_ref)
    rt.rt_render_batch_noalloc([j.struct() for j in got], c_got.data_ptr(), rt.make_opts(skip_empty=skip))
    torch.cuda.synchronize()
    for a, b in zip(ref, got):
        assert torch.equal(a.out, b.out)
        assert torch.equal(a.pixel_counts, b.pixel_counts)
    assert int(c_ref.item()) == int(c_got.item()) > 0
    return int(c_got.item())


def test_noalloc_batch_matches_render_batch(rt):
    import torch
    dims, sp = (96, 96, 64), (0.9, 0.9, 1.2)
    v = W.phantom_brain(31, dims=dims, spacing=sp)
    vol = rt.Volume(v, sp, storage=rt.U12)
    tf = rt.TransferFunction(W.random_tf(4096, 32, alpha_max=0.05), 0, 4095)
    cams = W.orbit_cameras(dims, sp, 36)
    print("noalloc: 36 views of 96x96x64 u12 at 160x160", flush=True)
    n1 = _run_pair(rt, torch, vol, tf, cams, 160)
    print("noalloc: 5 views at 72x72 (smaller second call)", flush=True)
    n2 = _run_pair(rt, torch, vol, tf, cams[3:8], 72)
    assert 0 < n2 < n1
    print("noalloc: 64 views (the limit) with empty-space skipping", flush=True)
    _run_pair(rt, torch, vol, tf, (cams + cams)[:64], 48, skip=True)
    print("noalloc: 65 views refused", flush=True)
    jobs = _jobs(rt, torch, vol, tf, (cams + cams)[:65], 16)
    with pytest.raises(rt.Unsupported):
        rt.rt_render_batch_noalloc([j.struct() for j in jobs])
    torch.cuda.synchronize()
    assert all(bool((j.out == -1.0).all()) for j in jobs)   # nothing was rendered
