"""The native serving runtime (rt_serve.h) on the GPU, through the C ABI.

Every served image must equal, bit for bit, the image rt_render gives for the
same request alone: in a mixed stream of volumes, image sizes, tables of
different sizes and ray functions; under an image pool so small that requests
wait for memory (first come, first served); with several client threads
calling at once; and after requests fail or the server shuts down with work
queued.
"""
import time

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


@pytest.fixture(scope="module")
def vols():
    sp = (0.9, 0.9, 1.2)
    return [(W.phantom_brain(201, dims=(96, 80, 64), spacing=sp), sp),
            (W.phantom_brain(202, dims=(128, 128, 80), spacing=sp), sp)]


def alone(rt, torch, srv, req):
    v = srv.volumes[req.volume_id]
    tf = rt.TransferFunction(req.tf_rgba, req.vmin, req.vmax)
    img = rt.render(v, tf, req.camera, req.width, req.height, req.step_vox, req.alpha_cutoff, req.bg,
                    ray_function=req.ray_function, iso_value=req.iso_value, iso_high=req.iso_high)
    torch.cuda.synchronize()
    return img


def make_requests(rt, vols, n, seed):
    from paper_1211_5595_amd.serve import RenderRequest
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        vi = int(rng.integers(0, len(vols)))
        dims = vols[vi][0].shape[::-1]
        cam = W.random_camera(rng, dims, vols[vi][1])
        side = int(rng.choice([17, 64, 100, 160]))
        K = int(rng.choice([64, 512, 4096]))
        fn = [rt.COMPOSITE, rt.COMPOSITE, rt.MIP, rt.THRESHOLD, rt.ISO][k % 5]
        lo = float(rng.uniform(500, 1500))
        out.append(RenderRequest(vi, cam, side, side + 3, W.random_tf(K, 900 + k, alpha_max=0.2), 0.0, 4095.0,
                                 float(rng.uniform(0.4, 1.0)), 0.99, (0.0, 0.1, 0.2, 0.3), None, fn, lo, lo + 800.0))
    return out


def test_mixed_stream_bitwise_equal_alone(rt, torch_mod, vols):
    from paper_1211_5595_amd.serve import NativeServer
    torch = torch_mod
    srv = NativeServer(64 << 20, n_streams=3, max_batch=16, storage=rt.U12)
    for i, (v, sp) in enumerate(vols):
        srv.add_volume(i, v, sp)
    reqs = make_requests(rt, vols, 60, 5)
    tickets = [srv.submit(r) for r in reqs]
    imgs = [srv.result(t, r.width, r.height) for t, r in zip(tickets, reqs)]
    st = srv.stats()
    assert st.submitted == 60 and st.completed == 60 and st.failed == 0 and st.pool_in_use == 0
    for r, img in zip(reqs, imgs):
        assert torch.equal(img, alone(rt, torch, srv, r))
    srv.close()


def test_requests_arriving_during_a_render_share_the_next_launch(rt, torch_mod, vols):
    """One stream: ten small requests submitted while a large render runs go
    out together in the next launch."""
    from paper_1211_5595_amd.serve import NativeServer, RenderRequest
    torch = torch_mod
    srv = NativeServer(128 << 20, n_streams=1, max_batch=16, storage=rt.U12, skip_empty=False)
    srv.add_volume(0, *vols[1])
    cams = W.orbit_cameras(vols[1][0].shape[::-1], vols[1][1], 11)
    big = RenderRequest(0, cams[0], 2048, 2048, W.random_tf(4096, 1, alpha_max=0.01), 0.0, 4095.0, 0.2, 1.0)
    small = [RenderRequest(0, c, 48, 40, W.random_tf(256, 10 + k), 0.0, 4095.0) for k, c in enumerate(cams[1:])]
    tb = srv.submit(big)
    ts = [srv.submit(r) for r in small]
    info_big = srv.wait(tb)
    infos = [srv.wait(t) for t in ts]
    assert info_big.state == rt.REQ_DONE and all(i.state == rt.REQ_DONE for i in infos)
    assert max(i.batch_size for i in infos) >= 5
    assert min(i.t_launch for i in infos) >= info_big.t_launch
    for t, r in zip(ts, small):
        img = srv.image(srv.wait(t), r.width, r.height).clone()
        torch.cuda.synchronize()
        assert torch.equal(img, alone(rt, torch, srv, r))
        srv.release(t)
    srv.release(tb)
    srv.close()


def test_small_pool_first_come_first_served(rt, torch_mod, vols):
    """A pool of two 100x103 images: the rest wait for memory, are launched in
    submission order, and the pool never holds more than its size."""
    from paper_1211_5595_amd.serve import NativeServer, RenderRequest
    torch = torch_mod
    img_bytes = (100 * 103 * 16 + 255) // 256 * 256
    srv = NativeServer(2 * img_bytes, n_streams=2, max_batch=8, storage=rt.U12)
    srv.add_volume(0, *vols[0])
    cams = W.orbit_cameras(vols[0][0].shape[::-1], vols[0][1], 12)
    reqs = [RenderRequest(0, c, 100, 103, W.random_tf(256, 40 + k, alpha_max=0.1), 0.0, 4095.0)
            for k, c in enumerate(cams)]
    tickets = [srv.submit(r) for r in reqs]
    infos, imgs = [], []
    for t, r in zip(tickets, reqs):
        info = srv.wait(t)
        assert info.state == rt.REQ_DONE
        infos.append((info.t_submit, info.t_launch, info.t_done))
        imgs.append(srv.image(info, r.width, r.height).clone())
        torch.cuda.synchronize()
        srv.release(t)
    launches = [x[1] for x in infos]
    assert launches == sorted(launches)
    assert all(a <= b <= c for a, b, c in infos)
    st = srv.stats()
    assert st.pool_peak <= 2 * img_bytes and st.pool_in_use == 0
    for r, img in zip(reqs, imgs):
        assert torch.equal(img, alone(rt, torch, srv, r))
    srv.close()


def test_rejections_and_ticket_rules(rt, torch_mod, vols):
    from paper_1211_5595_amd.serve import NativeServer, RenderRequest
    counter = torch_mod.zeros(1, dtype=torch_mod.int64, device="cuda")
    srv = NativeServer(1 << 20, n_streams=1, max_batch=4, storage=rt.U12, sample_counter=counter)
    srv.add_volume(0, *vols[0])
    cam = W.orbit_cameras(vols[0][0].shape[::-1], vols[0][1], 4)[1]
    tf = W.random_tf(128, 3)
    with pytest.raises(rt.OutOfMemory):          # larger than the whole pool
        srv.submit(RenderRequest(0, cam, 512, 512, tf))
    with pytest.raises(rt.InvalidArgument):      # eye == centre
        srv.submit(RenderRequest(0, W.Camera(cam.center, cam.center, cam.up, True, 30.0, 1.0), 32, 32, tf))
    with pytest.raises(rt.InvalidArgument):      # table out of [0, 1]
        srv.submit(RenderRequest(0, cam, 32, 32, tf * 2.0 + 0.5))
    with pytest.raises(rt.InvalidArgument):      # unbuilt ray function
        srv.submit(RenderRequest(0, cam, 32, 32, tf, ray_function=9))
    other = rt.Volume(vols[0][0], vols[0][1], storage=rt.U16)
    srv.volumes["u16"] = other
    with pytest.raises(rt.InvalidArgument):      # another storage type than the server's
        srv.submit(RenderRequest("u16", cam, 32, 32, tf))
    t = srv.submit(RenderRequest(0, cam, 32, 32, tf))
    info = srv.wait(t)
    assert info.state == rt.REQ_DONE and info.batch_size == 1
    # the server's batches counted into the caller's device counter: as rt_render counts the same view
    torch_mod.cuda.synchronize()
    ref = torch_mod.zeros(1, dtype=torch_mod.int64, device="cuda")
    rt.render(srv.volumes[0], rt.TransferFunction(tf, 0.0, 4095.0), cam, 32, 32, sample_counter=ref, skip_empty=True)
    torch_mod.cuda.synchronize()
    assert int(counter.item()) == int(ref.item()) > 0
    srv.release(t)
    with pytest.raises(rt.InvalidArgument):      # released: unknown
        srv.release(t)
    with pytest.raises(rt.InvalidArgument):
        srv.wait(t, 0.0)
    srv.close()


def test_shutdown_finishes_work_and_fails_what_cannot_run(rt, torch_mod, vols):
    """close() finishes queued and running requests; requests that can never
    be admitted because unreleased images hold the pool are failed, not
    waited for."""
    from paper_1211_5595_amd import rt_server_destroy
    from paper_1211_5595_amd.serve import NativeServer, RenderRequest
    img_bytes = (64 * 64 * 16 + 255) // 256 * 256
    srv = NativeServer(img_bytes, n_streams=1, max_batch=4, storage=rt.U12)
    srv.add_volume(0, *vols[1])
    cams = W.orbit_cameras(vols[1][0].shape[::-1], vols[1][1], 3)
    ts = [srv.submit(RenderRequest(0, c, 64, 64, W.random_tf(64, 8))) for c in cams]
    first = srv.wait(ts[0])
    assert first.state == rt.REQ_DONE
    time.sleep(0.05)                              # the others wait for the pool the first one holds
    assert srv.wait(ts[1], 0.0).state == rt.REQ_QUEUED
    h, srv.handle = srv.handle, None
    t0 = time.perf_counter()
    rt_server_destroy(h)
    assert time.perf_counter() - t0 < 5.0

    srv2 = NativeServer(8 << 20, n_streams=2, max_batch=2, storage=rt.U12)
    srv2.add_volume(0, *vols[1])
    for k in range(20):
        srv2.submit(RenderRequest(0, cams[k % 3], 128, 96, W.random_tf(256, k)))
    srv2.close()                                  # returns once all 20 have rendered


def test_concurrent_clients(rt, torch_mod, vols):
    """Four client threads submit, wait for and release their own requests at
    the same time (the C calls run without the interpreter lock), through a
    pool that holds only some of the images at once: every image equals the
    request rendered alone and the counters balance."""
    import threading

    from paper_1211_5595_amd.serve import NativeServer
    torch = torch_mod
    srv = NativeServer(4 << 20, n_streams=3, max_batch=8, storage=rt.U12)
    for i, (v, sp) in enumerate(vols):
        srv.add_volume(i, v, sp)
    per = [make_requests(rt, vols, 30, 60 + c) for c in range(4)]
    out = [[None] * 30 for _ in range(4)]
    errors = []

    def client(c):
        try:
            tickets = []
            for k, r in enumerate(per[c]):
                tickets.append(srv.submit(r))
                if k % 4 == 3:  # collect in bursts, oldest first
                    while tickets:
                        j = k + 1 - len(tickets)
                        out[c][j] = srv.result(tickets.pop(0), per[c][j].width, per[c][j].height)
            for j in range(30 - len(tickets), 30):
                out[c][j] = srv.result(tickets.pop(0), per[c][j].width, per[c][j].height)
        except Exception as e:  # reported by the main thread
            errors.append(e)

    threads = [threading.Thread(target=client, args=(c,)) for c in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads), "a client thread did not finish"
    assert not errors, errors
    st = srv.stats()
    assert st.submitted == 120 and st.completed == 120 and st.failed == 0
    assert st.pool_in_use == 0 and st.queued == 0 and st.running == 0
    assert st.pool_peak <= st.pool_bytes
    for c in range(4):
        for r, img in zip(per[c], out[c]):
            assert torch.equal(img, alone(rt, torch, srv, r))
    srv.close()
