"""The render server on the GPU: every served image equals the same request
rendered alone, bit for bit, while requests overlap on several streams under
a tight HBM budget."""
import time

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1211_5595_amd as rt
    from paper_1211_5595_amd.serve import GpuExecutor, RenderRequest, Server

    sp = (0.9, 0.9, 1.2)
    dims = {"a": (96, 80, 64), "b": (128, 128, 64)}
    ex = GpuExecutor(n_streams=3, max_batch=8)
    vols = {k: W.phantom_brain(21 + i, dims=d, spacing=sp) for i, (k, d) in enumerate(dims.items())}
    for k, v in vols.items():
        ex.add_volume(k, v, sp)
    budget = ex.resident_bytes() + 4 * 256 * 256 * 16 + 8 * 65536
    srv = Server(ex, budget_bytes=budget, max_batch=8)
    rng = np.random.default_rng(5)
    reqs = []
    for n in range(40):
        vid = "ab"[int(rng.integers(2))]
        side = int(rng.choice([64, 96, 128, 192, 256]))
        K = int(rng.choice([256, 1024, 4096]))
        reqs.append(RenderRequest(vid, W.random_camera(rng, dims[vid], sp), side, side,
                                  W.random_tf(K, 1000 + n, alpha_max=0.1), 0.0, 4095.0, 0.5, 0.99))
    srv.start()
    futs = []
    for r in reqs:
        futs.append(srv.submit(r))
        time.sleep(float(rng.exponential(2e-4)))
    srv.stop(drain=True)
    assert srv.peak_bytes <= budget
    assert srv.batches < len(reqs)                 # some requests were batched together
    for r, f in zip(reqs, futs):
        got = f.result(10.0)
        tf = rt.TransferFunction(r.tf_rgba, r.vmin, r.vmax)
        alone = rt.render(ex.volumes[r.volume_id], tf, r.camera, r.width, r.height, r.step_vox, r.alpha_cutoff)
        torch.cuda.synchronize()
        assert torch.equal(got, alone)
