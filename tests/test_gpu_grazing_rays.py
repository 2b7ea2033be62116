"""Rays that graze the volume's box (Section 4.1: a ray that misses the box
takes no samples and leaves the background; one that touches it is
composited).  The batched kernels and rt_render's single-view kernel set up
rays with the same float-float slab test, so every image and per-pixel sample
count of a batch plan equals rt_render's, bit for bit, on cameras whose rays
graze the box: image edges on the box faces, an eye on a face plane or inside
the box, a box a few pixels across, axis-aligned rays."""
import numpy as np
import pytest

import workloads as W
from workloads import Camera

pytestmark = pytest.mark.gpu

DIMS, SP = (96, 80, 48), (0.9, 1.1, 1.5)


def _cameras():
    c = W.box_center(DIMS, SP)
    hi = np.array([(n - 1) * s for n, s in zip(DIMS, SP)])
    R = W.bounding_radius(DIMS, SP)
    cams = []
    # orthographic down -z, the image's half-height exactly half the box's y extent:
    # the top and bottom pixel rows graze the y faces
    cams.append(Camera(tuple(c + [0, 0, 3 * R]), tuple(c), (0, 1, 0), False, 0.0, hi[1] / 2))
    # orthographic along +x, half-height slightly inside and slightly outside the box
    for f in (0.999999, 1.000001):
        cams.append(Camera(tuple(c - [3 * R, 0, 0]), tuple(c), (0, 0, 1), False, 0.0, f * hi[2] / 2))
    # eye on the x = 0 face plane looking along it, and on the y = hi face plane
    cams.append(Camera((0.0, c[1], c[2] + 2 * R), (0.0, c[1], c[2]), (0, 1, 0), True, 60.0))
    cams.append(Camera((c[0], hi[1], c[2] - 2 * R), (c[0], hi[1], c[2]), (1, 0, 0), True, 45.0))
    # eye inside the box
    cams.append(Camera(tuple(c + [1.0, -2.0, 0.5]), tuple(c + [10.0, 3.0, -4.0]), (0, 0, 1), True, 90.0))
    # the box a few pixels across, far away, oblique
    cams.append(Camera(tuple(c + 40 * R * np.array([0.6, -0.7, 0.4])), tuple(c), (0, 0, 1), True, 3.0))
    # the box's silhouette on tile edges: perspective fitting the bounding sphere, axis-aligned
    D = 3 * R
    fov = float(np.degrees(2 * np.arcsin(R / D)))
    cams.append(Camera(tuple(c + [0, -D, 0]), tuple(c), (0, 0, 1), True, fov))
    cams.append(Camera(tuple(c + [0, 0, D]), tuple(c), (0, 1, 0), True, fov))
    return cams


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1211_5595_amd as rt
    rt.lib()
    return rt


@pytest.mark.parametrize("skip", [False, True])
@pytest.mark.parametrize("layout", ["QUADS", "CELLS"])
def test_grazing_rays_batch_equals_single_view(rt, layout, skip):
    import torch
    g = W.phantom_brain(700, dims=DIMS, spacing=SP)
    vol = rt.Volume(g, SP, storage=rt.U12, layout=getattr(rt, "LAYOUT_" + layout))
    tf = rt.TransferFunction(W.random_tf(4096, 701, alpha_max=0.05), 0.0, 4095.0)
    cams = _cameras()
    sides = [(257, 131), (128, 128), (64, 200), (130, 66), (96, 96), (200, 150), (33, 45), (128, 128), (128, 128)]
    jobs = [rt.Job(vol, tf, cam, w, h, 0.5, 0.99, skip_empty=skip,
                   pixel_counts=torch.zeros((h, w), dtype=torch.int32, device="cuda"))
            for cam, (w, h) in zip(cams, sides)]
    plan = rt.BatchPlan(len(jobs), rt.U12, layout=getattr(rt, "LAYOUT_" + layout), skip_empty=skip, batch_form=1)
    plan.launch(jobs)
    torch.cuda.synchronize()
    hits = 0
    for k, j in enumerate(jobs):
        counts = torch.zeros_like(j.pixel_counts)
        img = rt.render(vol, tf, j.camera, j.width, j.height, 0.5, 0.99, skip_empty=skip, pixel_counts=counts)
        torch.cuda.synchronize()
        assert torch.equal(img, j.out), (k, j.camera)
        assert torch.equal(counts, j.pixel_counts), (k, j.camera)
        hits += int((counts > 0).sum())
    plan.close()
    assert hits > 0
