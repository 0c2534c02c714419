"""Host-side checks of planned batches and of the per-class tile tuner.

A plan is built on the host from image descriptors (fake device pointers
here: planning never touches the device), so its layout can be checked
without a GPU: one launch per level and tile configuration in use, a tile ->
image map covering every image's tile grid exactly once, and run-time
validation of the host copy before anything is launched."""
import ctypes
import json
import struct

import pytest

from paper_1705_08266_amd import _lib, autotune
import paper_1705_08266_amd as dwt

FAKE = 0x10000000
HEADER = struct.Struct("<Ii6iQ")          # magic, version, n, levels, inverse, dtype, wavelet,
LAUNCH = struct.Struct("<6i3Q")           # nlaunch, bytes; level, tile, f32 flags, images,
                                          # total, offsets of map, starts, params


def _images(sizes, levels):
    lib = _lib.load()
    arr = (_lib.Image * len(sizes))()
    base = FAKE
    for i, (w, h) in enumerate(sizes):
        px = w * h * 4
        ws = lib.dwt2_workspace_bytes(w, h, levels, 0)
        arr[i] = _lib.Image(base, w, base + px, w, base + 2 * px if ws else None, ws, w, h)
        base += 2 * px + ws + 4096
    return arr


def _plan(sizes, levels, inverse=0, class_tiles=None, flags=0):
    lib = _lib.load()
    imgs = _images(sizes, levels)
    ct = None if class_tiles is None else (ctypes.c_int32 * 4)(*class_tiles)
    n = ctypes.c_size_t()
    st = lib.dwt2_batch_plan_bytes(imgs, len(sizes), 0, 0, levels, inverse, 0, ct, flags,
                                   ctypes.byref(n))
    assert st == 0, st
    buf = (ctypes.c_ubyte * n.value)()
    assert lib.dwt2_batch_plan(imgs, len(sizes), 0, 0, levels, inverse, 0, ct, flags, buf,
                               n.value) == 0
    assert lib.dwt2_batch_plan(imgs, len(sizes), 0, 0, levels, inverse, 0, ct, flags, buf,
                               n.value - 1) == _lib.ERR_WORKSPACE
    return bytes(buf)


def _tiles_of(w, h, tile, wavelet="cdf97"):
    cfg = dwt.tile_configs(wavelet)[tile]
    ox, oy = cfg[4], cfg[5]
    nqx, nqy = w // 2, h // 2
    return (-(-nqx // ox)) * (-(-nqy // oy))


def _parse(plan):
    magic, version, n, levels, inverse, dtype, wavelet, nlaunch, nbytes = HEADER.unpack_from(plan)
    launches = [LAUNCH.unpack_from(plan, HEADER.size + k * LAUNCH.size) for k in range(nlaunch)]
    return dict(magic=magic, n=n, levels=levels, inverse=inverse, nlaunch=nlaunch,
                bytes=nbytes), launches


@pytest.mark.parametrize("inverse", [0, 1])
def test_plan_is_one_launch_per_level_with_a_complete_tile_map(inverse):
    sizes = [(64, 96), (256, 128), (1024, 512), (96, 64), (4096, 128), (512, 512)]
    L = 3
    plan = _plan(sizes, L, inverse)
    h, launches = _parse(plan)
    assert h["magic"] == 0x42545744 and h["n"] == len(sizes) and h["bytes"] == len(plan)
    assert h["nlaunch"] == L
    order = [l[0] for l in launches]
    assert order == (list(range(L, 0, -1)) if inverse else list(range(1, L + 1)))
    for (level, tile, fa, fb, images, total, off_img, off_start, off_params) in launches:
        assert tile == 0 and images == len(sizes)
        assert off_img % 256 == 0 and off_start % 256 == 0 and off_params % 256 == 0
        img = struct.unpack_from(f"<{total}i", plan, off_img)
        start = struct.unpack_from(f"<{images}i", plan, off_start)
        # every image's tiles form one contiguous run, in image order, of the
        # size its tile grid has at this level
        expect = [_tiles_of(w >> (level - 1), h >> (level - 1), tile) for w, h in sizes]
        assert total == sum(expect)
        pos = 0
        for i, cnt in enumerate(expect):
            assert start[i] == pos
            assert img[pos:pos + cnt] == (i,) * cnt
            pos += cnt


def test_plan_splits_a_level_by_tile_configuration():
    sizes = [(64, 64), (1024, 1024), (128, 96), (2048, 1024)]   # classes 0, 2, 0, 2
    plan = _plan(sizes, 1, class_tiles=[2, 1, 3, 0])
    h, launches = _parse(plan)
    assert h["nlaunch"] == 2
    assert sorted((l[1], l[4]) for l in launches) == [(2, 2), (3, 2)]
    lib = _lib.load()
    total = ctypes.c_int32()
    per = (ctypes.c_int32 * 1)()
    assert lib.dwt2_batch_launches(plan, len(plan), ctypes.byref(total), per) == 0
    assert total.value == 2 and per[0] == 2


def test_run_validates_the_host_plan_before_launching():
    lib = _lib.load()
    plan = bytearray(_plan([(64, 64), (128, 64)], 2))
    buf = (ctypes.c_ubyte * len(plan)).from_buffer(plan)
    E, U = _lib.ERR_INVALID_ARG, _lib.ERR_UNSUPPORTED
    assert lib.dwt2_batch_run(buf, len(plan) - 8, FAKE, 0, 0, None) == E      # wrong size
    assert lib.dwt2_batch_run(buf, len(plan), None, 0, 0, None) == E           # no device copy
    assert lib.dwt2_batch_run(buf, len(plan), FAKE, 7, 0, None) == U           # scheme
    assert lib.dwt2_batch_run(buf, len(plan), FAKE, 0, 4, None) == U           # unknown flag
    bad = bytearray(plan)
    bad[0] ^= 1                                                                 # magic
    assert lib.dwt2_batch_run((ctypes.c_ubyte * len(bad)).from_buffer(bad), len(bad), FAKE, 0,
                              0, None) == E
    bad = bytearray(plan)
    LAUNCH.pack_into(bad, HEADER.size, 1, 99, 1, 1, 2, 4, 256, 512, 768)       # tile id 99
    assert lib.dwt2_batch_run((ctypes.c_ubyte * len(bad)).from_buffer(bad), len(bad), FAKE, 0,
                              0, None) == E


def test_plan_rejects_bad_batches():
    lib = _lib.load()
    n = ctypes.c_size_t()
    imgs = _images([(64, 64)], 1)
    assert lib.dwt2_batch_plan_bytes(imgs, 0, 0, 0, 1, 0, 0, None, 0, ctypes.byref(n)) == \
        _lib.ERR_INVALID_ARG                                                   # no images
    assert lib.dwt2_batch_plan_bytes(imgs, 1, 0, 0, 1, 2, 0, None, 0, ctypes.byref(n)) == \
        _lib.ERR_UNSUPPORTED                                                   # direction
    ct = (ctypes.c_int32 * 4)(0, 0, 0, 17)
    assert lib.dwt2_batch_plan_bytes(imgs, 1, 0, 0, 1, 0, 0, ct, 0, ctypes.byref(n)) == \
        _lib.ERR_UNSUPPORTED                                                   # tile id
    imgs = _images([(64, 64)], 1)
    assert lib.dwt2_batch_plan_bytes(imgs, 1, 0, 0, 7, 0, 0, None, 0, ctypes.byref(n)) == \
        _lib.ERR_INVALID_ARG                                                   # 64 % 128


# ---- the tuner, with an injected timer (no GPU) ----------------------------------
def test_tune_picks_each_class_argmin_and_caches(tmp_path):
    calls = []
    table = {0: {0: 3.0, 1: 1.0, 2: 2.0}, 1: {0: 1.0, 1: 5.0, 2: 0.5},
             2: {0: 0.2, 1: 0.3, 2: 0.4}, 3: {0: 9.0, 1: 8.0, 2: 7.0}}

    def timer(cls, tile):
        calls.append((cls, tile))
        return table[cls][tile]

    cache = tmp_path / "tune.json"
    got = autotune.tune("cdf97", "nonseparable", "f32", 3, cache_path=str(cache), timer=timer,
                        candidates=[0, 1, 2], device_name="dev")
    assert got == [1, 2, 0, 2]
    # every class is timed on its own, once per candidate
    assert sorted(calls) == [(c, t) for c in range(4) for t in range(3)]
    data = json.loads(cache.read_text())
    assert data["dev|cdf97|nonseparable|f32|L3"]["class_tiles"] == [1, 2, 0, 2]
    # second call: from the cache, no timing
    calls.clear()
    assert autotune.tune("cdf97", "nonseparable", "f32", 3, cache_path=str(cache), timer=timer,
                         candidates=[0, 1, 2], device_name="dev") == [1, 2, 0, 2]
    assert calls == []
    # another key is tuned afresh; force re-tunes
    table[0][0] = 0.1
    assert autotune.tune("cdf97", "nonseparable", "f16", 3, cache_path=str(cache), timer=timer,
                         candidates=[0, 1, 2], device_name="dev")[0] == 0
    calls.clear()
    assert autotune.tune("cdf97", "nonseparable", "f32", 3, cache_path=str(cache), timer=timer,
                         candidates=[0, 1, 2], device_name="dev", force=True)[0] == 0
    assert len(calls) == 12


def test_tune_default_candidates_are_the_compiled_configurations():
    seen = set()
    autotune.tune(timer=lambda c, t: seen.add(t) or float(t), device_name="dev")
    assert seen == {c[0] for c in dwt.tile_configs("cdf97")}


# Head tile grids of the 12-wavefront, 4-row head: a forward tile owns 58 x 18
# level-2 quads, an inverse tile 116 x 44 level-1 quads.
def _head_tiles(w, h, inverse):
    if inverse:
        return (-(-(w // 2) // 116)) * (-(-(h // 2) // 44))
    return (-(-(w // 4) // 58)) * (-(-(h // 4) // 18))


@pytest.mark.parametrize("inverse", [0, 1])
def test_head_plan_fuses_levels_one_and_two(inverse):
    sizes = [(64, 96), (256, 128), (1024, 512), (96, 64), (4096, 128), (512, 512), (32, 32)]
    L = 3
    plan = _plan(sizes, L, inverse, flags=_lib.PLAN_HEAD)
    h, launches = _parse(plan)
    assert h["nlaunch"] == L - 1
    assert [l[0] for l in launches] == ([3, 1] if inverse else [1, 3])
    head = [l for l in launches if l[1] == _lib.TILE_HEAD]
    assert len(head) == 1
    level, tile, fa, fb, images, total, off_img, off_start, off_params = head[0]
    assert level == 1 and images == len(sizes) and (fa, fb) == (1, 1)
    img = struct.unpack_from(f"<{total}i", plan, off_img)
    start = struct.unpack_from(f"<{images}i", plan, off_start)
    expect = [_head_tiles(w, hh, inverse) for w, hh in sizes]
    assert total == sum(expect)
    pos = 0
    for i, cnt in enumerate(expect):
        assert start[i] == pos and img[pos:pos + cnt] == (i,) * cnt
        pos += cnt
    lib = _lib.load()
    n = ctypes.c_int32()
    per = (ctypes.c_int32 * L)()
    assert lib.dwt2_batch_launches(plan, len(plan), ctypes.byref(n), per) == 0
    assert n.value == L - 1 and list(per) == [1, 0, 1]


def test_head_flag_changes_nothing_with_one_level_and_unknown_flags_are_refused():
    sizes = [(64, 64), (256, 128)]
    assert _plan(sizes, 1, flags=_lib.PLAN_HEAD) == _plan(sizes, 1)
    lib = _lib.load()
    n = ctypes.c_size_t()
    assert lib.dwt2_batch_plan_bytes(_images(sizes, 2), 2, 0, 0, 2, 0, 0, None, 2,
                                     ctypes.byref(n)) == _lib.ERR_UNSUPPORTED


def test_run_refuses_a_head_launch_off_level_one():
    lib = _lib.load()
    plan = bytearray(_plan([(64, 64), (128, 64)], 2, flags=_lib.PLAN_HEAD))
    h, launches = _parse(bytes(plan))
    assert [l[1] for l in launches] == [_lib.TILE_HEAD]
    bad = bytearray(plan)
    LAUNCH.pack_into(bad, HEADER.size, 2, *launches[0][1:])                    # level 2
    assert lib.dwt2_batch_run((ctypes.c_ubyte * len(bad)).from_buffer(bad), len(bad), FAKE, 0,
                              0, None) == _lib.ERR_INVALID_ARG
