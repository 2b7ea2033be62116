"""The uneven batch at its full size, in the launch the benchmark times: 32
seeded phantoms of four sizes (up to 512x512x256) as 12-bit halves in quad
bricks, 128 random views of 256^2..1024^2 pixels, one batch plan over all of
them.  Sampled pixels of every view against the FP64 oracle (tie-aware,
1e-5, sample counts exact off ties; arXiv:1211.5595, Sections 3.2 and
4.1-4.2), every image bitwise equal to the same plan over the cell layout and
to the empty-space-skipping form."""
import numpy as np
import pytest

import workloads as W

from test_gpu_parity import DELTA, check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1211_5595_amd as rt
    rt.lib()
    return rt


def test_uneven_batch_full_size(rt, orc):
    import torch
    specs, views = W.random_views(seed=4)
    grids, quads, tfs, tf_np = [], [], [], []
    for i, sp in enumerate(specs):
        v = W.phantom_brain(sp.seed, dims=sp.dims, spacing=sp.spacing)
        grids.append(v)
        quads.append(rt.Volume(v, sp.spacing, storage=rt.U12, layout=rt.LAYOUT_QUADS))
        tf_np.append(W.random_tf(4096, 1000 + i, alpha_max=0.05))
        tfs.append(rt.TransferFunction(tf_np[-1], 0.0, 4095.0))
    print(f"{len(specs)} volumes ready", flush=True)
    counts = [torch.zeros((s, s), dtype=torch.int32, device="cuda") for _, _, s in views]
    jobs = [rt.Job(quads[vi], tfs[vi], cam, s, s, 0.5, 0.99, pixel_counts=c)
            for (vi, cam, s), c in zip(views, counts)]
    plan = rt.BatchPlan(len(jobs), rt.U12, layout=rt.LAYOUT_QUADS)
    counter = torch.zeros(1, dtype=torch.int64, device="cuda")
    plan.launch(jobs, sample_counter=counter)
    torch.cuda.synchronize()
    assert int(counter.item()) == sum(int(c.to(torch.int64).sum()) for c in counts)
    # the timed (non-counting) form, and the skipping form, bitwise equal
    timed = [rt.Job(quads[vi], tfs[vi], cam, s, s, 0.5, 0.99) for vi, cam, s in views]
    plan.launch(timed)
    skip = [rt.Job(quads[vi], tfs[vi], cam, s, s, 0.5, 0.99, skip_empty=True) for vi, cam, s in views]
    plan_s = rt.BatchPlan(len(jobs), rt.U12, layout=rt.LAYOUT_QUADS, skip_empty=True)
    plan_s.launch(skip)
    torch.cuda.synchronize()
    for a, b, c in zip(jobs, timed, skip):
        assert torch.equal(a.out, b.out) and torch.equal(a.out, c.out)
    del skip, plan_s
    # sampled pixels of every view against the oracle, one volume at a time
    rng = np.random.default_rng(404)
    worst = 0.0
    for vi, sp in enumerate(specs):
        ov, otf = orc.Volume(grids[vi], sp.spacing), orc.TF(tf_np[vi], 0.0, 4095.0)
        for k, (vj, cam, s) in enumerate(views):
            if vj != vi:
                continue
            px = rng.choice(s * s, size=256, replace=False)
            ref = orc.render(ov, otf, cam, s, s, 0.5, 0.99, pixels=px, tie_delta=DELTA, want_band=True)
            got = timed[k].out.cpu().numpy().astype(np.float64).reshape(-1, 4)[px]
            w, _ = check(got, ref, counts[k].cpu().numpy().reshape(-1)[px], f"volume {vi} {sp.dims} view {k}")
            worst = max(worst, w)
        del ov, otf
    print(f"128 views sampled: worst band distance {worst:.3g}", flush=True)
    # the same plan over the cell layout: bitwise equal images
    del quads, jobs
    cells = [rt.Volume(v, sp.spacing, storage=rt.U12) for v, sp in zip(grids, specs)]
    cjobs = [rt.Job(cells[vi], tfs[vi], cam, s, s, 0.5, 0.99) for vi, cam, s in views]
    rt.BatchPlan(len(cjobs), rt.U12).launch(cjobs)
    torch.cuda.synchronize()
    for a, b in zip(timed, cjobs):
        assert torch.equal(a.out, b.out)
