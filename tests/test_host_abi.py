"""Host-only checks of the C ABI: exports, decomposition, arena sizing, validation.

No call here touches a GPU: every function used is pure host code, or fails
validation before any device work.
"""
import os
import re

import numpy as np
import pytest

from paper_2202_11819_amd import j3d

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "j3d.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"^\s*(?:j3d_status|const char \*)\s*(j3d_\w+)\s*\(", text, flags=re.M))


def test_library_exports_every_declared_symbol():
    declared = _declared_functions()
    assert len(declared) >= 30
    for name in declared:
        assert hasattr(j3d._lib, name), name
    assert declared == set(j3d.EXPORTED)


def test_version_and_no_error():
    assert "gfx950" in j3d.j3d_version()


# ---- decomposition (Sec. IV-A: surface-minimising split) -------------------------

def _paper_rows():
    rows = []
    with open(os.path.join(GOLDEN, "paper_memory_sizes.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                edge, gpus, sx, sy, sz, nbytes = line.split()
                rows.append((int(edge), int(gpus), (int(sx), int(sy), int(sz)), float(nbytes)))
    return rows


@pytest.mark.parametrize("row", _paper_rows())
def test_paper_node_split_and_memory(row):
    edge, gpus, split, paper_bytes = row
    assert j3d.j3d_auto_split((edge,) * 3, gpus) == split
    nb, ext = j3d.j3d_block_extents(j3d.Problem((edge,) * 3, None, auto_parts=gpus))
    assert nb == split
    blk = tuple(e[0] for e in ext)
    assert all(len(set(e)) == 1 for e in ext)  # even split
    # two copies of one GPU's block (interior cells); the paper says "roughly"
    two_fields = 2 * 8 * blk[0] * blk[1] * blk[2]
    assert 0.95 * paper_bytes <= two_fields <= 1.1 * paper_bytes
    # the library's fields add halo storage only
    fb = j3d.j3d_field_bytes(j3d.Problem(blk))
    assert two_fields < fb < 1.1 * two_fields


def test_auto_split_prefers_small_surface():
    assert j3d.j3d_auto_split((64, 64, 64), 1) == (1, 1, 1)
    assert j3d.j3d_auto_split((64, 64, 64), 8) == (2, 2, 2)
    assert j3d.j3d_auto_split((512, 512, 512), 512) == (8, 8, 8)
    assert j3d.j3d_auto_split((1000, 10, 10), 4) == (4, 1, 1)
    with pytest.raises(j3d.J3DError) as e:
        j3d.j3d_auto_split((2, 2, 2), 27)
    assert e.value.status == j3d.J3D_EINVAL
    # more parts than a problem may have blocks: rejected at once, not searched
    for parts in ((1 << 22) + 1, 2**31 - 1):
        with pytest.raises(j3d.J3DError) as e:
            j3d.j3d_auto_split((1 << 30,) * 3, parts)
        assert e.value.status == j3d.J3D_EINVAL
    assert j3d.j3d_auto_split((1 << 30,) * 3, 1 << 21) == (1 << 7,) * 3


def test_block_extents_rules():
    nb, ext = j3d.j3d_block_extents(j3d.Problem((10, 7, 5), None, auto_parts=6))
    assert nb == (3, 2, 1)
    assert ext == ([4, 3, 3], [4, 3], [5])
    nb, ext = j3d.j3d_block_extents(j3d.Problem((12, 6, 9), (3, 2, 3)))
    assert ext == ([4, 4, 4], [3, 3], [3, 3, 3])
    nb, ext = j3d.j3d_block_extents(j3d.Problem((10, 6, 9), (3, 1, 2), split=([1, 2, 7], None, [8, 1])))
    assert ext == ([1, 2, 7], [6], [8, 1])


@pytest.mark.parametrize("kwargs", [
    dict(n=(0, 4, 4)),
    dict(n=(4, 4, 4), nblk=(5, 1, 1)),
    dict(n=(10, 4, 4), nblk=(3, 1, 1)),                       # even split does not divide
    dict(n=(10, 4, 4), nblk=(2, 1, 1), split=([3, 6], None, None)),  # sum mismatch
    dict(n=(10, 4, 4), nblk=(2, 1, 1), split=([0, 10], None, None)),  # empty block
    dict(n=(4, 4, 4), nblk=(1, 0, 1)),
    dict(n=(4, 4, 4), bc=(0, 0, float("nan"), 0, 0, 0)),
    dict(n=(4, 4, 4), bc=(0, 0, 0, float("inf"), 0, 0)),
    dict(n=(2 ** 31, 1, 1)),
    dict(n=(4096, 4096, 4096)),                              # one block beyond 2^31 cells
    dict(n=(20000, 20000, 1)),                               # one x-y plane beyond 2^28 cells
])
def test_invalid_problems_are_rejected(kwargs):
    p = j3d.Problem(kwargs.pop("n"), **kwargs)
    for fn in (j3d.j3d_arena_bytes, j3d.j3d_field_bytes, j3d.j3d_block_extents):
        with pytest.raises(j3d.J3DError) as e:
            fn(p)
        assert e.value.status == j3d.J3D_EINVAL
    assert j3d.j3d_last_error() != ""


def test_arena_covers_fields_and_grows():
    small = j3d.Problem((64, 64, 64))
    over = j3d.Problem((64, 64, 64), (4, 4, 4))
    for p in (small, over):
        assert j3d.j3d_arena_bytes(p) > j3d.j3d_field_bytes(p) >= 2 * 8 * 64 ** 3
        assert j3d.j3d_arena_bytes(p) % 4096 == 0
    assert j3d.j3d_arena_bytes(over) > j3d.j3d_arena_bytes(small)
    # 512^3 as 8^3 blocks: two fields of 1.07 GB plus halo storage (~9% at 64^3 blocks)
    cfg1 = j3d.Problem((512, 512, 512), (8, 8, 8))
    fb = j3d.j3d_field_bytes(cfg1)
    assert 2 * 8 * 512 ** 3 < fb < 1.1 * 2 * 8 * 512 ** 3
    assert j3d.j3d_batch_arena_bytes([small, over]) > j3d.j3d_arena_bytes(over)


def test_variant_table():
    vs = j3d.variants()
    assert len(vs) >= 8
    flat = 0
    for tx, ty, threads in vs:
        assert threads % 64 == 0 and threads <= 1024
        if tx == 0:  # flattened: ty is the cell capacity, a whole number of cells per thread
            flat += 1
            assert threads >= 256 and ty % threads == 0
        else:
            assert tx % 32 == 0 and 32 <= tx <= 256 and ty >= 16
    assert flat >= 1
    with pytest.raises(j3d.J3DError):
        j3d.j3d_variant_info(len(vs))


def test_pool_sizing_host_only():
    p = j3d.Problem((32, 40, 48))
    b = j3d.j3d_pool_request_bytes(p)
    assert b >= 2 * 8 * 32 * 40 * 48 and b % 4096 == 0
    assert j3d.j3d_pool_overhead_bytes(256) > 0
    with pytest.raises(j3d.J3DError) as e:
        j3d.j3d_pool_request_bytes(j3d.Problem((64, 64, 64), (2, 1, 1)))
    assert e.value.status == j3d.J3D_EINVAL
    with pytest.raises(j3d.J3DError):
        j3d.j3d_pool_overhead_bytes(0)


def test_create_validates_before_device_work():
    p = j3d.Problem((16, 16, 16), (2, 2, 2))
    need = j3d.j3d_arena_bytes(p)
    with pytest.raises(j3d.J3DError) as e:
        j3d.j3d_create(p, 0, need, 0)                 # NULL arena
    assert e.value.status == j3d.J3D_EINVAL
    with pytest.raises(j3d.J3DError) as e:
        j3d.j3d_create(p, 0x10000 + 8, need, 0)       # misaligned
    assert e.value.status == j3d.J3D_EINVAL
    with pytest.raises(j3d.J3DError) as e:
        j3d.j3d_create(p, 0x10000, need - 4096, 0)    # arena too small
    assert e.value.status == j3d.J3D_ENOMEM
    with pytest.raises(j3d.J3DError) as e:
        j3d.j3d_batch_create([p], [-1], 0x10000, 1 << 40, 0)
    assert e.value.status == j3d.J3D_EINVAL


def test_two_sweep_entry_points_validate_handles():
    # NULL handles are rejected before any device work
    for fn, args in ((j3d._lib.j3d_batch_run_two_sweep, (None, None)), (j3d._lib.j3d_pool_set_two_sweep, (None, 1)),
                     (j3d._lib.j3d_run, (None, 2, 9, None))):
        assert fn(*args) == j3d.J3D_EINVAL
    assert j3d.MODES["two_sweep"] == 9


def _no_gpu_here():
    if os.path.exists("/dev/kfd"):
        return False
    try:
        import torch
        return torch.cuda.device_count() == 0
    except Exception:
        return True


@pytest.mark.skipif(not _no_gpu_here(), reason="only meaningful where no GPU is present")
def test_create_without_device_is_edevice():
    p = j3d.Problem((8, 8, 8))
    with pytest.raises(j3d.J3DError) as e:
        j3d.j3d_create(p, 0x10000, j3d.j3d_arena_bytes(p), 0)
    assert e.value.status == j3d.J3D_EDEVICE
    with pytest.raises(j3d.J3DError) as e:
        j3d.j3d_device_cus()
    assert e.value.status == j3d.J3D_EDEVICE


def test_pool_entry_points_validate_before_device_work():
    # every pool call rejects a NULL handle or bad arguments with EINVAL (or
    # ENOMEM for a short arena) before it touches a device: none is present here
    import ctypes
    L = j3d._lib
    i32, i64, dbl = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_double()
    u64 = ctypes.c_uint64()
    buf = (ctypes.c_double * 64)()
    for fn, args in ((L.j3d_pool_fetch, (None, 0, buf, ctypes.byref(dbl), ctypes.byref(i64))),
                     (L.j3d_pool_fetch, (None, 0, None, None, None)),
                     (L.j3d_pool_result, (None, 0, ctypes.byref(dbl), ctypes.byref(i64))),
                     (L.j3d_pool_admit, (None, None, 10, 0.0, 0, None, ctypes.byref(i32))),
                     (L.j3d_pool_step, (None, 1)),
                     (L.j3d_pool_poll, (None, None, 0, ctypes.byref(i32), None)),
                     (L.j3d_pool_release, (None, 0)),
                     (L.j3d_pool_usage, (None, None, None)),
                     (L.j3d_pool_set_policy, (None, 0, 1, 0)),
                     (L.j3d_pool_set_tune, (None, None)),
                     (L.j3d_pool_destroy, (None,)),
                     (L.j3d_pool_overhead_bytes, (0, ctypes.byref(u64))),
                     (L.j3d_pool_overhead_bytes, (4, None))):
        assert fn(*args) == j3d.J3D_EINVAL, fn.__name__
    h = ctypes.c_void_p()
    over = j3d.j3d_pool_overhead_bytes(4)
    aligned, unaligned = 1 << 20, (1 << 20) + 8
    cases = [((None, over + 4096, 4096, 4, None, ctypes.byref(h)), j3d.J3D_EINVAL),        # NULL arena
             ((unaligned, over + 4096, 4096, 4, None, ctypes.byref(h)), j3d.J3D_EINVAL),   # unaligned
             ((aligned, over + 4096, 4096, 0, None, ctypes.byref(h)), j3d.J3D_EINVAL),     # no slots
             ((aligned, over + 4096, 0, 4, None, ctypes.byref(h)), j3d.J3D_EINVAL),        # no budget
             ((aligned, over + 4095, 4096, 4, None, ctypes.byref(h)), j3d.J3D_ENOMEM),     # short arena
             ((aligned, over + 4096, 4096, 4, None, None), j3d.J3D_EINVAL)]                # NULL out
    for args, want in cases:
        assert L.j3d_pool_create(*args) == want, args
    assert not h.value  # no handle was made
    # a decomposed problem is not a pool request
    with pytest.raises(j3d.J3DError) as e:
        j3d.j3d_pool_request_bytes(j3d.Problem((64, 64, 64), (2, 1, 1)))
    assert e.value.status == j3d.J3D_EINVAL


def test_flattened_tile_shapes_fit_their_variants(tmp_path):
    # the shape rule shared by the planner and the kernel, checked exhaustively
    # on the host (widths 1..1200, heights 1..700, every thread count / capacity)
    import subprocess
    exe = tmp_path / "flat_shape_check"
    src = os.path.join(ROOT, "tests", "flat_shape_check.cpp")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_2202_11819_amd", "csrc"),
                           "-I", os.path.join(ROOT, "include"), src, "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout[-2000:]
    assert " 0 bad" in out.stdout


def test_xcd_ranges_partition_each_launch(tmp_path):
    # the per-XCD tile ranges of a one-workgroup-per-tile launch: in order,
    # equal work within one tile, every tile run exactly once by the grid
    import subprocess
    exe = tmp_path / "xcd_split_check"
    src = os.path.join(ROOT, "tests", "xcd_split_check.cpp")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_2202_11819_amd", "csrc"),
                           "-I", os.path.join(ROOT, "include"), src, "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout[-2000:]
    assert " 0 bad" in out.stdout


def test_fused_halo_sources_link_neighbours(tmp_path):
    # the per-block halo sources the fused sweep reads: each equals the
    # neighbour formula it replaces, -1 without a neighbour, and a lone block
    # built from a zeroed descriptor (the pool's requests) reads its own ghosts
    import subprocess
    exe = tmp_path / "halo_link_check"
    src = os.path.join(ROOT, "tests", "halo_link_check.cpp")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_2202_11819_amd", "csrc"),
                           "-I", os.path.join(ROOT, "include"), src, "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout[-2000:]
    assert " 0 bad" in out.stdout


def test_tile_tables_cover_every_cell_once(tmp_path):
    # the planner's sweep tiles, from the built library: inside the block,
    # within the variant's shape and z-chunk, every cell exactly once, for
    # every variant on ragged and aligned block shapes
    import subprocess
    pkg = os.path.join(ROOT, "paper_2202_11819_amd")
    exe = tmp_path / "tile_cover_check"
    src = os.path.join(ROOT, "tests", "tile_cover_check.cpp")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                           "-I", os.path.join(pkg, "csrc"), "-I", os.path.join(ROOT, "include"), src,
                           "-o", str(exe), "-L", pkg, "-lj3d", f"-Wl,-rpath,{pkg}"])
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout[-2000:]
    assert " 0 bad" in out.stdout
