"""The quad-brick layout (16-bit and 12-bit storage in 2/3 of the cell
layout's memory, one 16-byte load per sample): its relayout bit for bit
against the bricks built on the host, images bit for
bit equal to the cell layout of the same storage type (single views, batches,
empty-space skipping, every ray function), and against the FP64 oracle on
brain views and random grids with large steps (arXiv:1211.5595, Sections 3.2
and 4.1-4.2: the same trilinear samples and compositing, only the storage
differs)."""
import numpy as np
import pytest

import workloads as W

from test_gpu_parity import DELTA, check, gpu_render

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
def brain(rt, orc):
    dims, sp = (256, 256, 160), (0.9, 0.9, 1.2)
    v = W.phantom_brain(11)
    t = W.random_tf(4096, 12, alpha_max=0.05)
    return dict(np=v, dims=dims, sp=sp, gtf=rt.TransferFunction(t, 0, 4095), ov=orc.Volume(v, sp),
                otf=orc.TF(t, 0, 4095), cams=W.orbit_cameras(dims, sp, 36))


def _quads_on_host(v, h12):
    """[z][y][x] source -> the quad bricks as 16-bit words: bricks [bz][by][bx] of 2x2
    padded cell columns (x = 2 bx + (c & 1), y = 2 by + (c >> 1)) by 4 padded layers
    (z = 3 bz + l), [c][l][4] within a brick, x fastest within a quad; every index
    clamped into the volume after the one-node border shift."""
    nz, ny, nx = v.shape
    nbx, nby, nbz = (nx + 2) // 2, (ny + 2) // 2, (nz + 3) // 3
    x = 2 * np.arange(nbx)[:, None] + np.array([0, 1])[None, :]          # [bx][dx]
    y = 2 * np.arange(nby)[:, None] + np.array([0, 1])[None, :]          # [by][dy]
    z = 3 * np.arange(nbz)[:, None] + np.arange(4)[None, :]              # [bz][l]
    zi = np.clip(z - 1, 0, nz - 1)
    g = v.astype(np.int64)
    out = np.zeros((nbz, nby, nbx, 2, 2, 4, 4), dtype=np.int64)          # [bz][by][bx][dy][dx][l][q]
    for q, (ox, oy) in enumerate(((-1, -1), (0, -1), (-1, 0), (0, 0))):
        xi = np.clip(x + ox, 0, nx - 1)
        yi = np.clip(y + oy, 0, ny - 1)
        # g[zi][:, :, yi][..., xi] -> [bz][l][by][dy][bx][dx]
        s = g[zi][:, :, yi][:, :, :, :, xi]
        out[..., q] = s.transpose(0, 2, 4, 3, 5, 1)
    if h12:
        return (np.minimum(out, 4096) - 2048).astype(np.float16).view(np.uint16)
    return out.astype(np.uint16)


@pytest.mark.parametrize("storage", ["U16", "U12"])
def test_quads_relayout_bit_exact(rt, torch_mod, storage):
    rng = np.random.default_rng(301)
    for dims in ((2, 2, 2), (17, 5, 9), (40, 33, 21)):
        v = rng.integers(0, 5000, size=dims[::-1], dtype=np.uint16)
        gv = rt.Volume(v, (1.0, 1.2, 0.8), storage=getattr(rt, storage), layout=rt.LAYOUT_QUADS)
        torch_mod.cuda.synchronize()
        want = np.ascontiguousarray(_quads_on_host(v, storage == "U12")).reshape(-1)
        got = gv.buf.cpu().numpy()[: want.size * 2].view(np.uint16)
        assert np.array_equal(got, want), (storage, dims)


@pytest.mark.parametrize("storage", ["U16", "U12"])
def test_quads_brain_views_match_cells_and_oracle(rt, torch_mod, orc, brain, storage):
    st = getattr(rt, storage)
    gx = rt.Volume(brain["np"], brain["sp"], storage=st, layout=rt.LAYOUT_QUADS)
    gc = rt.Volume(brain["np"], brain["sp"], storage=st)
    for view in (5, 23):
        cam = brain["cams"][view]
        got, c = gpu_render(rt, torch_mod, gx, brain["gtf"], cam, 512, 512, 0.5, 0.99)
        cel, cc = gpu_render(rt, torch_mod, gc, brain["gtf"], cam, 512, 512, 0.5, 0.99)
        assert np.array_equal(got, cel) and np.array_equal(c, cc)
        ref = orc.render(brain["ov"], brain["otf"], cam, 512, 512, 0.5, 0.99, tie_delta=DELTA, want_band=True)
        check(got, ref, c, f"{storage} quads brain view {view}")


def test_quads_batches_skipping_and_ray_functions_bitwise(rt, torch_mod, brain):
    """The 36-view orbit as one plan, with and without empty-space skipping,
    and the other ray functions: quads equal to cells bit for bit."""
    torch = torch_mod
    gx = rt.Volume(brain["np"], brain["sp"], storage=rt.U12, layout=rt.LAYOUT_QUADS)
    gc = rt.Volume(brain["np"], brain["sp"], storage=rt.U12)
    cams = brain["cams"]
    for skip in (False, True):
        px = rt.BatchPlan(36, rt.U12, layout=rt.LAYOUT_QUADS, skip_empty=skip)
        pc = rt.BatchPlan(36, rt.U12, skip_empty=skip)
        jx = [rt.Job(gx, brain["gtf"], c, 256, 256, 0.5, 0.99, skip_empty=skip) for c in cams]
        jc = [rt.Job(gc, brain["gtf"], c, 256, 256, 0.5, 0.99, skip_empty=skip) for c in cams]
        px.launch(jx)
        pc.launch(jc)
        torch.cuda.synchronize()
        for a, b in zip(jx, jc):
            assert torch.equal(a.out, b.out), skip
    for fn, lo, hi, top in ((rt.MIP, 0.0, 0.0, 4095.0), (rt.XRAY, 0.0, 0.0, 4095.0 * 150), (rt.AVERAGE, 0.0, 0.0, 4095.0),
                            (rt.ISO, 1000.0, 0.0, 4095.0), (rt.THRESHOLD, 1200.0, 2600.0, 4095.0)):
        tf = rt.TransferFunction(W.random_tf(4096, 12, alpha_max=0.05), 0, top)
        a = rt.render(gx, tf, cams[3], 200, 160, ray_function=fn, iso_value=lo, iso_high=hi)
        b = rt.render(gc, tf, cams[3], 200, 160, ray_function=fn, iso_value=lo, iso_high=hi)
        torch.cuda.synchronize()
        assert torch.equal(a, b), fn


@pytest.mark.parametrize("seed", range(6))
def test_quads_random_grids_large_steps(rt, torch_mod, orc, seed):
    """Ragged grids, random cameras, steps up to 6 voxels (the request after a
    ray's last sample then lands far outside the grid and is capped): both
    storages against the oracle."""
    rng = np.random.default_rng(3100 + seed)
    dims = tuple(int(x) for x in rng.integers(2, 60, 3))
    sp = tuple(float(x) for x in rng.uniform(0.4, 2.5, 3))
    v = rng.integers(0, 4097, size=dims[::-1], dtype=np.uint16)
    v = ((v.astype(np.int64) + np.roll(v, 1, 0) + np.roll(v, 1, 1)) // 3).astype(np.uint16)
    t = W.random_tf(int(rng.integers(64, 4097)), seed + 310, alpha_max=float(rng.uniform(0.05, 0.9)))
    cam = W.random_camera(rng, dims, sp)
    Wd, Hd = int(rng.integers(1, 120)), int(rng.integers(1, 100))
    step = float(rng.choice([0.3, 0.7, 2.5, 6.0])) if seed < 4 else float(rng.uniform(0.2, 1.2))
    cutoff = float(rng.uniform(0.6, 1.0))
    gtf = rt.TransferFunction(t, 0, 4096)
    ref = orc.render(orc.Volume(v, sp), orc.TF(t, 0, 4096), cam, Wd, Hd, step, cutoff, tie_delta=DELTA,
                     want_band=True)
    for storage in ("U16", "U12"):
        gv = rt.Volume(v, sp, storage=getattr(rt, storage), layout=rt.LAYOUT_QUADS)
        got, c = gpu_render(rt, torch_mod, gv, gtf, cam, Wd, Hd, step, cutoff)
        check(got, ref, c, f"{storage} quads seed {seed} dims {dims} step {step}")
        out = rt.render_batch([rt.Job(gv, gtf, cam, Wd, Hd, step, cutoff)])[0]
        torch_mod.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().astype(np.float64), got)


@pytest.fixture(scope="module")
def largest_quads(rt, orc):
    """The largest grid of the quad-brick layout in one axis pair: 1022 x 1022
    x 188 nodes, 512 x 512 x 63 bricks of 128 bytes, one z-brick short of
    2^31 bytes (byte offsets up to 2^31 - 2^25): a separable smooth field
    plus separable integer noise on a 12-bit range, and the oracle's view."""
    dims, sp = (1022, 1022, 188), (1.0, 1.0, 1.0)
    ax = [np.arange(n, dtype=np.float32) for n in dims]
    smooth = (np.sin(ax[2] / 13.0 + 0.5)[:, None, None] * np.cos(ax[1] / 41.0)[None, :, None]
              * (1500.0 * np.sin(ax[0] / 37.0)).astype(np.float32)[None, None, :])
    hrng = np.random.default_rng(82)
    hz, hy, hx = (hrng.integers(0, 81, size=n).astype(np.int16) for n in dims[::-1])
    noise = (hz[:, None, None] + hy[None, :, None]) + hx[None, None, :]
    v = (np.rint(smooth).astype(np.int16) + (noise % 81 - 40) + 2048).astype(np.uint16)
    del smooth, noise
    return dims, sp, v, orc.Volume(v, sp)


@pytest.mark.parametrize("storage", ["U12", "U16"])
def test_quads_largest_volume(rt, torch_mod, orc, largest_quads, storage):
    """Rays through the far corner of the largest quad-brick grid (where the
    byte offsets approach 2^31) and through the whole volume, from one launch
    and from a batch, against the oracle on sampled pixels."""
    torch = torch_mod
    dims, sp, v, ov = largest_quads
    st = getattr(rt, storage)
    nbytes = rt.rt_volume_bytes(dims, st, rt.LAYOUT_QUADS)
    assert (1 << 31) - (1 << 26) <= nbytes < (1 << 31)
    gv = rt.Volume(v, sp, storage=st, layout=rt.LAYOUT_QUADS)
    t = W.random_tf(4096, 34, alpha_max=0.05)
    gtf, otf = rt.TransferFunction(t, 0, 4095), orc.TF(t, 0, 4095)
    hi = np.array([(n - 1) * s for n, s in zip(dims, sp)])
    corner = W.Camera(tuple(hi + np.array([90.0, 70.0, 40.0])), tuple(hi - np.array([60.0, 60.0, 30.0])), (0, 0, 1),
                      True, 40.0)
    # and the whole volume from above (an orbit about z would see this flat box edge-on)
    c = hi / 2
    above = W.Camera(tuple(c + np.array([300.0, -400.0, 1200.0])), tuple(c), (0, 1, 0), True, 50.0)
    cams = [corner, above]
    rng = np.random.default_rng(83)
    for ci, cam in enumerate(cams):
        got, c = gpu_render(rt, torch, gv, gtf, cam, 192, 160, 0.5, 0.99)
        out = rt.render_batch([rt.Job(gv, gtf, cam, 192, 160, 0.5, 0.99)])[0]
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().astype(np.float64), got)
        assert (c > 0).mean() > 0.3
        px = rng.choice(192 * 160, size=400, replace=False)
        ref = orc.render(ov, otf, cam, 192, 160, 0.5, 0.99, pixels=px, tie_delta=DELTA, want_band=True)
        check(got.reshape(-1, 4)[px], ref, c.reshape(-1)[px], f"{storage} largest quad volume, camera {ci}")
    del gv
    torch.cuda.empty_cache()
