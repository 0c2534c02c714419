"""Host-side checks of the buffer-overlap rules of the C ABI.

Buffers of one call must not share a byte (outputs with inputs, outputs with
each other), and in batched calls no image or job may write a buffer that
another one reads or writes. The library tests strided regions exactly when
they share a pitch (the bands of one Mallat array interleave within rows),
so these tests compare its answer with a brute-force byte-set overlap on
small layouts. Pointers are fake and never dereferenced: every call either
fails its checks or, with no GPU present, fails at the launch."""
import ctypes

import numpy as np
import pytest

from paper_1705_08266_amd import _lib

FAKE = 0x10000000
E, W = _lib.ERR_INVALID_ARG, _lib.ERR_WORKSPACE


def _bytes(off, rows, cols, pitch, es=4):
    return {off + r * pitch * es + c for r in range(rows) for c in range(cols * es)}


def _no_gpu():
    try:
        import torch
        return torch.cuda.device_count() == 0
    except Exception:       # noqa: BLE001 - no torch: no GPU either
        return True


def test_multi_level_overlap_matches_brute_force():
    """src and coef of a forward: refused exactly when they share a byte
    (same pitch), never accepted when they do (any pitch)."""
    lib = _lib.load()
    rng = np.random.default_rng(7)
    for _ in range(600):
        w, h = 8, int(rng.choice([4, 8]))
        ps, pc = w + int(rng.integers(0, 9)), w + int(rng.integers(0, 9))
        if rng.random() < 0.6:
            pc = ps
        so, co = 4 * int(rng.integers(0, 64)), 4 * int(rng.integers(0, 64))
        sd = _lib.Desc(w, h, ps, _lib.F32)
        cd = _lib.Desc(w, h, pc, _lib.F32)
        st = lib.dwt2_forward(FAKE + so, ctypes.byref(sd), FAKE + co, ctypes.byref(cd),
                              0, 2, 0, 0, None, 0, None)
        brute = bool(_bytes(so, h, w, ps) & _bytes(co, h, w, pc))
        assert st in (E, W)
        if brute:
            assert st == E, (so, co, ps, pc)
        elif ps == pc:
            assert st == W, (so, co, ps, pc)


def test_side_by_side_views_are_accepted():
    """Two W x H views of one 2W-wide buffer (same pitch) do not overlap."""
    lib = _lib.load()
    d = _lib.Desc(64, 64, 128, _lib.F32)
    assert lib.dwt2_forward(FAKE, ctypes.byref(d), FAKE + 64 * 4, ctypes.byref(d),
                            0, 2, 0, 0, None, 0, None) == W
    assert lib.dwt2_forward(FAKE, ctypes.byref(d), FAKE + 32 * 4, ctypes.byref(d),
                            0, 2, 0, 0, None, 0, None) == E


def _level(lib, full, ll, hl, lh, hh, pitch_b=64):
    # 64 x 64 FP32 level: bands 32 x 32
    return lib.dwt2_forward_level(full, 64, 0, 64, 64, ll, pitch_b, 0, hl, lh, hh, pitch_b, 0,
                                  0, 0, -1, None)


def test_level_outputs_must_not_overlap_each_other():
    lib = _lib.load()
    B = FAKE + (1 << 24)
    # hl and lh are the same buffer
    assert _level(lib, FAKE, B, B + 32 * 4, B + 32 * 4, B + 32 * 64 * 4 + 32 * 4) == E
    # ll shares its first row with hl (hl starts 16 columns into ll)
    assert _level(lib, FAKE, B, B + 16 * 4, B + 32 * 64 * 4, B + 32 * 64 * 4 + 32 * 4) == E
    # hh overlaps the input
    assert _level(lib, FAKE, B, B + 32 * 4, B + 32 * 64 * 4, FAKE + 100) == E


@pytest.mark.skipif(not _no_gpu(), reason="passes its checks and would launch on a GPU")
def test_level_mallat_views_pass_the_checks():
    """ll, hl, lh and hh as the four quadrants of one 64-pitch Mallat array
    interleave within rows yet share no byte: the checks pass and the call
    goes on to the launch (which fails here: no GPU)."""
    lib = _lib.load()
    B = FAKE + (1 << 24)
    st = _level(lib, FAKE, B, B + 32 * 4, B + 32 * 64 * 4, B + 32 * 64 * 4 + 32 * 4)
    assert st == _lib.ERR_HIP


def _image(src, dst, ws=None, wsb=0, w=64, h=64):
    return _lib.Image(src, w, dst, w, ws, wsb, w, h)


def _plan_status(imgs, levels=1, inverse=0):
    lib = _lib.load()
    n = ctypes.c_size_t()
    return lib.dwt2_batch_plan_bytes(imgs, len(imgs), 0, 0, levels, inverse, 0, None, 0,
                                     ctypes.byref(n))


def test_batch_images_must_not_share_outputs():
    lib = _lib.load()
    A, B, C = FAKE, FAKE + (1 << 24), FAKE + (2 << 24)
    # two images write the same coefficients
    assert _plan_status((_lib.Image * 2)(_image(A, C), _image(B, C))) == E
    # the second image writes the first one's input
    assert _plan_status((_lib.Image * 2)(_image(A, B), _image(C, A + 64))) == E
    # shared workspace
    need = lib.dwt2_workspace_bytes(64, 64, 2, 0)
    ws = FAKE + (3 << 24)
    imgs = (_lib.Image * 2)(_image(A, B, ws, need), _image(C, FAKE + (4 << 24), ws + 256, need))
    assert _plan_status(imgs, levels=2) == E


def test_batch_shared_input_is_allowed():
    """Two images may read the same source (planning is host-only)."""
    A = FAKE
    imgs = (_lib.Image * 2)(_image(A, FAKE + (1 << 24)), _image(A, FAKE + (2 << 24)))
    assert _plan_status(imgs) == _lib.OK
    assert _plan_status(imgs, inverse=1) == _lib.OK


def test_level_batch_jobs_must_not_race():
    lib = _lib.load()
    B = FAKE + (1 << 24)
    J = _lib.LevelJob

    def job(full, base):
        return J(full, 64, 0, base, 64, 0, base + 32 * 4, base + 32 * 64 * 4,
                 base + 32 * 64 * 4 + 32 * 4, 64, 0, 64, 64)
    # two forward jobs write the same bands
    jobs = (J * 2)(job(FAKE, B), job(FAKE + (2 << 24), B))
    assert lib.dwt2_forward_level_batch(jobs, 2, 0, 0, None, None) == E
    # an inverse job writes the image another job reads as its LL band
    jobs = (J * 2)(job(FAKE, B), job(FAKE + (3 << 24), FAKE + 4))
    assert lib.dwt2_inverse_level_batch(jobs, 2, 0, 0, None, None) == E
