"""The C ABI on the CPU: the library loads, exports every symbol declared in
include/rt.h, and its host-only paths (sizes, validation) behave as the
header documents.  No kernel is launched here."""
import ctypes as C
import os
import re

import pytest

from conftest import ROOT


@pytest.fixture(scope="module")
def rt():
    import paper_1211_5595_amd as rt
    if not os.path.exists(rt.LIB_PATH):
        from paper_1211_5595_amd import build
        build.build()
    rt.lib()
    return rt


def declared_functions():
    """Every function declared in the public headers (include/*.h)."""
    import glob
    names = set()
    for h in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))):
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names.update(re.findall(r"\b(rt_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_every_declared_symbol_is_exported(rt):
    names = declared_functions()
    assert len(names) >= 22 and "rt_server_submit" in names and "rt_render" in names
    L = rt.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_oracle_and_product_share_no_symbols(rt, orc):
    L = C.CDLL(orc.LIB_PATH)
    for n in declared_functions():
        assert not hasattr(L, n)


def skip_bytes(dims):
    """Skip-brick value ranges appended to every layout: bricks of 2^e padded
    cells (0..n per axis), the smallest e >= 3 with at most 65536 bricks,
    8 bytes each, rounded to 256; then the ranges of the super-bricks
    (ceil(bricks / 4) per axis), 8 bytes each, rounded to 256."""
    e = 3
    while True:
        per_axis = [(n + 1 + (1 << e) - 1) >> e for n in dims]
        nb = per_axis[0] * per_axis[1] * per_axis[2]
        if nb <= 65536:
            ns = 1
            for b in per_axis:
                ns *= (b + 3) // 4
            return (nb * 8 + 255) // 256 * 256 + (ns * 8 + 255) // 256 * 256
        e += 1


def test_skip_brick_counts():
    r = lambda x: (x + 255) // 256 * 256
    assert skip_bytes((256, 256, 160)) == r(33 * 33 * 21 * 8) + r(9 * 9 * 6 * 8)
    assert skip_bytes((512, 512, 256)) == r(33 * 33 * 17 * 8) + r(9 * 9 * 5 * 8)   # 16^3-cell bricks
    assert skip_bytes((2, 2, 2)) == 512


def test_volume_bytes(rt):
    r256 = lambda x: (x + 255) // 256 * 256

    def vb(dims, *a):
        return rt.rt_volume_bytes(dims, *a) - skip_bytes(dims)

    # linear: (n+2)^3 padded nodes times the element size, rounded to 256
    L = rt.LAYOUT_LINEAR
    assert vb((256, 256, 160), rt.U16, L) == ((258 * 258 * 162 * 2 + 255) // 256) * 256
    assert vb((64, 64, 32), rt.U8, L) == ((66 * 66 * 34 + 255) // 256) * 256
    assert vb((2, 2, 2), rt.F32, L) == 256
    # cells: padded cells 0..n per axis rounded up to 2x2x2 blocks, 8 corners each
    assert vb((256, 256, 160), rt.U16) == r256(129 * 129 * 81 * 8 * 8 * 2)
    assert vb((64, 64, 32), rt.U8) == r256(33 * 33 * 17 * 8 * 8)
    assert vb((2, 2, 2), rt.F32) == r256(2 * 2 * 2 * 8 * 8 * 4)
    # 15-bit difference cells: the same size as 16-bit cells
    assert vb((256, 256, 160), rt.U15) == r256(129 * 129 * 81 * 8 * 8 * 2)
    # 12-bit half cells: likewise
    assert vb((256, 256, 160), rt.U12) == r256(129 * 129 * 81 * 8 * 8 * 2)
    # polynomial cells (integer data): as cells, 8 binary32 coefficients each
    assert vb((256, 256, 160), rt.U16, rt.LAYOUT_POLY) == r256(129 * 129 * 81 * 8 * 8 * 4)
    assert vb((64, 64, 32), rt.U8, rt.LAYOUT_POLY) == r256(33 * 33 * 17 * 8 * 8 * 4)
    # quad bricks (16-bit and 12-bit storage): 2x2 padded cell columns (0..n) by 3 cells in z
    # per 128-byte brick
    X = rt.LAYOUT_QUADS
    assert vb((256, 256, 160), rt.U16, X) == r256(129 * 129 * 54 * 128)
    assert vb((256, 256, 160), rt.U12, X) == r256(129 * 129 * 54 * 128)
    assert vb((512, 512, 256), rt.U12, X) == r256(257 * 257 * 86 * 128)
    assert vb((2, 2, 2), rt.U16, X) == r256(2 * 2 * 1 * 128)
    assert vb((3, 3, 4), rt.U16, X) == r256(2 * 2 * 2 * 128)
    # the largest quad volume of 1022 x 1022 cross-section: 63 z-bricks, one short of 2^31 bytes
    assert vb((1022, 1022, 188), rt.U12, X) == 512 * 512 * 63 * 128
    with pytest.raises(rt.Unsupported):
        vb((1022, 1022, 189), rt.U12, X)
    # brick-scaled, halo bricks: ceil((n-1)/B) bricks per axis, (B+3)^3 codes and 8 bytes each
    nb = 16 * 16 * 10
    assert vb((256, 256, 160), rt.U8_BRICKSCALED, rt.LAYOUT_BRICKS, 16) == \
        r256(r256(nb * 8) + nb * 19 ** 3)
    # brick-scaled, cells: (n+1)//2+1 shifted blocks per axis, 64 B of codes and 8 B each,
    # then the per-brick parameters
    ncb = 129 * 129 * 81
    assert vb((256, 256, 160), rt.U8_BRICKSCALED, rt.LAYOUT_CELLS, 16) == \
        r256(r256(r256(ncb * 8) + ncb * 64) + nb * 8)


def test_cell_layout_size_limits(rt):
    """2^24 blocks of 2x2x2 cells at most, and block strides below 2^24: the
    largest accepted grids and the first refused ones."""
    for st, b in ((rt.U12, 128), (rt.U16, 128), (rt.F32, 256)):
        assert rt.rt_volume_bytes((508, 510, 510), st) >= 255 * 256 * 256 * b
        with pytest.raises(rt.Unsupported):
            rt.rt_volume_bytes((510, 510, 510), st)
    rt.rt_volume_bytes((4092, 2046, 2), rt.U16)           # 8 * 2047 * 1024 < 2^24
    with pytest.raises(rt.Unsupported):
        rt.rt_volume_bytes((4094, 2046, 2), rt.U16)       # 8 * 2048 * 1024 = 2^24


@pytest.mark.parametrize("dims,storage,layout,brick,exc", [
    ((1, 4, 4), 1, 0, 0, "InvalidArgument"),
    ((4, 4, 4), 4, 0, 12, "InvalidArgument"),
    ((4, 4, 4), 1, 0, 8, "InvalidArgument"),
    ((4, 4, 4), 1, 2, 0, "InvalidArgument"),
    ((4, 4, 4), 4, 1, 8, "InvalidArgument"),
    ((2048, 2048, 1024), 1, 0, 0, "Unsupported"),
    ((4, 4, 4), 9, 0, 0, "InvalidArgument"),
    ((5000, 5000, 4), 1, 1, 0, "Unsupported"),
    ((4, 4, 4), 2, 3, 0, "InvalidArgument"),    # polynomial layout: integer storage only
    ((4, 4, 4), 3, 3, 0, "InvalidArgument"),
    ((4, 4, 4), 4, 3, 8, "InvalidArgument"),
    ((4, 4, 4), 5, 1, 0, "InvalidArgument"),    # 15-bit difference cells: cell layout only
    ((4, 4, 4), 5, 3, 0, "InvalidArgument"),
    ((4, 4, 4), 6, 1, 0, "InvalidArgument"),    # 12-bit halves: cells or quad bricks only
    ((4, 4, 4), 6, 3, 0, "InvalidArgument"),
    ((4, 4, 4), 7, 0, 0, "InvalidArgument"),
    ((4, 4, 4), 0, 4, 0, "InvalidArgument"),    # quads: 16-bit and 12-bit storage only
    ((4, 4, 4), 2, 4, 0, "InvalidArgument"),
    ((4, 4, 4), 3, 4, 0, "InvalidArgument"),
    ((4, 4, 4), 4, 4, 8, "InvalidArgument"),
    ((4, 4, 4), 5, 4, 0, "InvalidArgument"),
    ((4, 4, 4), 1, 5, 0, "InvalidArgument"),    # no layout 5
    ((2048, 2046, 2), 1, 4, 0, "Unsupported"),   # 2^20 quad bricks per z-brick slice or more
    ((1024, 1024, 1024), 6, 4, 0, "Unsupported"),  # quads of 2 GiB or more
    ((2, 2, 65534), 1, 4, 0, "Unsupported"),      # more than 65533 slices
])
def test_volume_bytes_errors(rt, dims, storage, layout, brick, exc):
    with pytest.raises(getattr(rt, exc)):
        rt.rt_volume_bytes(dims, storage, layout, brick)


def test_tf_and_workspace_bytes(rt):
    # table (256-aligned) then K+2 int32 running counts (256-aligned)
    assert rt.rt_tf_bytes(4096) == 65536 + 16640 and rt.rt_tf_bytes(2) == 512
    for K in (1, 4097):
        with pytest.raises(rt.InvalidArgument):
            rt.rt_tf_bytes(K)
    assert rt.rt_batch_workspace_bytes(1) < rt.rt_batch_workspace_bytes(128)
    with pytest.raises(rt.InvalidArgument):
        rt.rt_batch_workspace_bytes(0)


def test_null_arguments_are_reported_not_fatal(rt):
    L = rt.lib()
    dims = (C.c_int64 * 3)(4, 4, 4)
    assert L.rt_render(None, dims, None, None, None, 8, 8, 0.5, 0.99, None, None, None, None) == 1
    assert b"NULL" in L.rt_last_error()
    h = C.c_void_p()
    sp = (C.c_double * 3)(1, 1, 1)
    assert L.rt_create_volume(None, 1, dims, sp, 1, 0, 0, None, 0, None, C.byref(h)) == 1
    assert L.rt_render_batch(None, 0, None, 0, None, None, None) == 1
    # one job past the largest batch is refused before the jobs are looked at
    over = (rt.rt_render_job * 4097)()
    assert L.rt_render_batch(over, 4097, C.c_void_p(4096), 1 << 30, None, None, None) == 4
    assert b"too many jobs" in L.rt_last_error()
    assert L.rt_batch_plan_launch(None, None, 0, None, None) == 1
    assert L.rt_destroy_volume(None) == 0 and L.rt_destroy_tf(None) == 0 and L.rt_batch_plan_destroy(None) == 0
    assert L.rt_status_string(2) == b"buffer too small"
    assert L.rt_version().startswith(b"rtvol")


def test_launch_options_are_checked_before_any_device_work(rt):
    """Tile shape, wavefronts per block and tile order are validated first."""
    L = rt.lib()
    dims = (C.c_int64 * 3)(4, 4, 4)
    for kw, code in ((dict(tile_order=3), 1), (dict(tile_order=-1), 1), (dict(tile=(3, 21)), 4),
                     (dict(tile=(16, 8)), 4), (dict(waves_per_block=3), 4)):
        o = rt.make_opts(**kw)
        assert L.rt_render(None, dims, None, None, None, 8, 8, 0.5, 0.99, None, None, C.byref(o), None) == code, kw
    # fixed-step batches take at most 12 wavefronts per workgroup, batches with skipping 16
    jobs = (rt.rt_render_job * 1)()
    o = rt.make_opts(waves_per_block=16)
    assert L.rt_render_batch(jobs, 1, C.c_void_p(4096), 1 << 30, None, C.byref(o), None) == 4
    assert b"at most 12" in L.rt_last_error()
    jobs[0].skip_empty = 1
    assert L.rt_render_batch(jobs, 1, C.c_void_p(4096), 1 << 30, None, C.byref(o), None) == 1  # shape accepted
    assert b"volume" in L.rt_last_error()
    o = rt.make_opts(waves_per_block=12)
    jobs[0].skip_empty = 0
    assert L.rt_render_batch(jobs, 1, C.c_void_p(4096), 1 << 30, None, C.byref(o), None) == 1


def test_product_path_does_not_import_oracle():
    """The product package never imports the oracle nor the generators."""
    pkg = os.path.join(ROOT, "paper_1211_5595_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src and "oracle.h" not in src, f
                assert "import workloads" not in src and "from workloads" not in src, f


def test_server_arena_and_argument_checks(rt):
    """The serving runtime's sizes, and its argument checks, which run before
    any device work."""
    r = lambda x: (x + 255) // 256 * 256
    lane = r(rt.rt_batch_workspace_bytes(64)) + 64 * r(rt.rt_tf_bytes(4096))
    assert rt.rt_server_arena_bytes(3, 64, 1 << 20) == 3 * lane + (1 << 20)
    assert rt.rt_server_arena_bytes(1, 1, 1000) == r(rt.rt_batch_workspace_bytes(1)) + r(rt.rt_tf_bytes(4096)) \
        + 1024
    for args in ((0, 4, 4096), (9, 4, 4096), (1, 0, 4096), (1, 257, 4096), (1, 4, 255)):
        with pytest.raises(rt.InvalidArgument):
            rt.rt_server_arena_bytes(*args)
    L = rt.lib()
    h = C.c_void_p()
    need = rt.rt_server_arena_bytes(2, 8, 1 << 20)
    cases = [((2, 8, 1, 0, None, None, need, 1 << 20), 1),        # NULL arena
             ((2, 8, 1, 0, None, 4096 + 16, need, 1 << 20), 1),   # misaligned arena
             ((2, 8, 1, 0, None, 4096, need - 1, 1 << 20), 2),    # arena too small
             ((2, 8, 12, 0, None, 4096, need, 1 << 20), 1),       # unknown storage
             ((2, 8, 6, 1, None, 4096, need, 1 << 20), 1),        # u12 exists in the cell layout only
             ((0, 8, 1, 0, None, 4096, need, 1 << 20), 1)]        # no stream
    for (ns, mb, st, lay, opts, arena, nbytes, pool), code in cases:
        assert L.rt_server_create(ns, mb, st, lay, opts, C.c_void_p(arena), nbytes, pool, C.byref(h)) == code
        assert h.value is None
    bad = rt.make_opts(tile_order=5)
    assert L.rt_server_create(2, 8, 1, 0, C.byref(bad), C.c_void_p(4096), need, 1 << 20, C.byref(h)) == 1
    assert L.rt_server_submit(None, None, None) == 1 and L.rt_server_release(None, 1) == 1
    assert L.rt_server_destroy(None) == 0


def test_struct_layouts_match_the_header(rt, tmp_path):
    """The ctypes mirrors of the ABI structs have the C compiler's sizes and
    field offsets (compiled from include/*.h with the host C compiler)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    structs = {"rt_camera": rt.rt_camera, "rt_render_opts": rt.rt_render_opts, "rt_render_job": rt.rt_render_job,
               "rt_request": rt.rt_request, "rt_request_info": rt.rt_request_info,
               "rt_server_stats": rt.rt_server_stats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rt_serve.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'    printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'    printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:-1]): int(l.split()[-1]) for l in out if l.strip()}
    for name, cls in structs.items():
        assert got[(name, "size")] == C.sizeof(cls), name
        for f, _ in cls._fields_:
            assert got[(name, f)] == getattr(cls, f).offset, (name, f)
