"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, and rejects bad arguments before enqueuing anything (no GPU needed:
every call here returns during argument checking)."""
import ctypes
import os
import re

import pytest

import paper_1705_08266_amd as dwt
from paper_1705_08266_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dwt2.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(dwt2_\w+)\s*\(", text)
    return sorted(set(names))


def test_library_is_built_and_loads():
    assert os.path.exists(_lib.LIB_PATH)
    lib = _lib.load()
    assert lib.dwt2_version() >= 100


def test_every_declared_symbol_is_exported_and_bound():
    names = _declared_functions()
    assert len(names) == len(_lib.SIGNATURES)
    lib = _lib.load()
    for n in names:
        assert hasattr(lib, n), n
        assert n in _lib.SIGNATURES, f"{n} missing from the Python binding"


# The boundary's core prototypes, written as the scope table states them
# (parameter names aside). Compiling them after the header makes the C
# compiler reject any difference in a parameter or return type.
SECTION_8B_PROTOTYPES = """
size_t      dwt2_workspace_bytes(int32_t width, int32_t height, int32_t levels, dwt2_dtype dtype);
int         dwt2_forward(const void* src, const dwt2_desc* src_d, void* coef, const dwt2_desc* coef_d,
                         dwt2_wavelet w, int32_t levels, dwt2_boundary b, dwt2_scheme s,
                         void* workspace, size_t workspace_bytes, hipStream_t stream);
int         dwt2_inverse(const void* coef, const dwt2_desc* coef_d, void* dst, const dwt2_desc* dst_d,
                         dwt2_wavelet w, int32_t levels, dwt2_boundary b, dwt2_scheme s,
                         void* workspace, size_t workspace_bytes, hipStream_t stream);
const char* dwt2_status_string(int status);
int         dwt2_last_hip_error(void);
"""


def test_header_matches_the_scope_prototypes(tmp_path):
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "proto.c"
    src.write_text('#include "dwt2.h"\n' + SECTION_8B_PROTOTYPES)
    r = subprocess.run([cc, "-std=c11", "-Wall", "-Werror", "-fsyntax-only",
                        "-I", os.path.dirname(HEADER), str(src)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    # a wrong prototype is rejected (the check above has teeth)
    bad = tmp_path / "bad.c"
    bad.write_text('#include "dwt2.h"\n'
                   "int dwt2_forward(const void*, const dwt2_desc*, void*, const dwt2_desc*,"
                   " dwt2_wavelet, int32_t, dwt2_boundary, dwt2_scheme, const int32_t*,"
                   " void*, size_t, void* const*, hipStream_t);\n")
    r = subprocess.run([cc, "-std=c11", "-fsyntax-only", "-I", os.path.dirname(HEADER),
                        str(bad)], capture_output=True, text=True)
    assert r.returncode != 0


def test_core_entry_points_take_the_scope_arguments():
    """dwt2_forward / dwt2_inverse take exactly the 11 arguments; tuning and
    timing hooks live in the _ex calls."""
    assert len(_lib.SIGNATURES["dwt2_forward"][1]) == 11
    assert len(_lib.SIGNATURES["dwt2_inverse"][1]) == 11
    assert len(_lib.SIGNATURES["dwt2_forward_ex"][1]) == 13
    assert len(_lib.SIGNATURES["dwt2_workspace_bytes"][1]) == 4


def test_workspace_bytes():
    lib = _lib.load()
    for dt in (_lib.F32, _lib.F16, _lib.BF16):     # intermediate LL is FP32 for every dtype
        assert lib.dwt2_workspace_bytes(64, 64, 1, dt) == 0
        assert lib.dwt2_workspace_bytes(64, 64, 2, dt) == 32 * 32 * 4
        assert lib.dwt2_workspace_bytes(64, 64, 3, dt) == (32 * 32 + 16 * 16) * 4
        assert lib.dwt2_workspace_bytes(4096, 4096, 5, dt) == (2048 * 2048 + 1024 * 1024) * 4
        assert lib.dwt2_workspace_bytes(48, 64, 5, dt) == 0      # 48 not divisible by 32
        assert lib.dwt2_workspace_bytes(64, 64, 0, dt) == 0
    assert lib.dwt2_workspace_bytes(64, 64, 2, 7) == 0          # unknown dtype


def test_tile_configs_cover_the_lifting_halo():
    for w, np_ in (("cdf97", 2), ("cdf53", 1)):
        cfgs = dwt.tile_configs(w)
        assert len(cfgs) >= 4
        for (t, qpl, rows, waves, ox, oy) in cfgs:   # one halo lane each side
            assert qpl >= np_
            assert ox == 64 * qpl - 2 * qpl
            assert oy == waves * rows - 2 * np_ > 0


def test_default_tile_is_valid():
    n = _lib.load().dwt2_tile_config_count()
    for (w, h) in ((4096, 4096), (256, 256), (2, 2), (16384, 64)):
        t = dwt.default_tile(w, h)
        assert 0 <= t < n
    assert dwt.default_tile(3, 4) == _lib.ERR_INVALID_ARG


def test_status_strings():
    lib = _lib.load()
    for s in (0, -1, -2, -3, -4, 17):
        assert lib.dwt2_status_string(s)


FAKE = 0x10000000       # never dereferenced: every call below fails its checks


def _fwd(src=FAKE, sd=None, dst=FAKE + (1 << 30), dd=None, wavelet=0, levels=1,
         boundary=0, scheme=0, tiles=None, ws=None, wsb=0):
    lib = _lib.load()
    sd = sd or _lib.Desc(64, 64, 64, _lib.F32)
    dd = dd or _lib.Desc(64, 64, 64, _lib.F32)
    if tiles is None:
        return lib.dwt2_forward(src, ctypes.byref(sd), dst, ctypes.byref(dd), wavelet, levels,
                                boundary, scheme, ws, wsb, None)
    return lib.dwt2_forward_ex(src, ctypes.byref(sd), dst, ctypes.byref(dd), wavelet, levels,
                               boundary, scheme, ws, wsb, tiles, None, None)


def test_forward_argument_errors():
    E, U, W = _lib.ERR_INVALID_ARG, _lib.ERR_UNSUPPORTED, _lib.ERR_WORKSPACE
    assert _fwd(src=None) == E
    assert _fwd(dst=None) == E
    assert _fwd(levels=0) == E
    assert _fwd(levels=17) == E
    assert _fwd(levels=7) == E                                   # 64 % 128 != 0
    assert _fwd(wavelet=5) == U
    assert _fwd(scheme=9) == U
    assert _fwd(boundary=1) == U
    assert _fwd(sd=_lib.Desc(64, 64, 32, _lib.F32)) == E         # pitch < width
    assert _fwd(dd=_lib.Desc(64, 32, 64, _lib.F32)) == E         # shape mismatch
    assert _fwd(dd=_lib.Desc(64, 64, 64, _lib.F16)) == E         # dtype mismatch
    assert _fwd(sd=_lib.Desc(64, 64, 64, 7), dd=_lib.Desc(64, 64, 64, 7)) == U
    assert _fwd(dst=FAKE + 64) == E                              # overlap
    assert _fwd(levels=2) == W                                   # no workspace
    assert _fwd(levels=2, ws=FAKE + (2 << 30), wsb=100) == W     # too small
    assert _fwd(levels=2, ws=FAKE + 4, wsb=1 << 20) == E         # workspace overlaps
    bad = (ctypes.c_int32 * 1)(99)
    assert _fwd(tiles=bad) == U
    assert _fwd(sd=_lib.Desc(66, 64, 66, _lib.F32), dd=_lib.Desc(66, 64, 66, _lib.F32),
                levels=2) == E                                   # 66 % 4 != 0


def test_fused_tail_tile_ids():
    """DWT2_TILE_TAIL must mark a suffix of 2..DWT2_TAIL_MAX levels."""
    U, W, T = _lib.ERR_UNSUPPORTED, _lib.ERR_WORKSPACE, _lib.TILE_TAIL

    def tiles(*ids):
        return (ctypes.c_int32 * len(ids))(*ids)

    assert _fwd(levels=3, tiles=tiles(T, 1, T)) == U          # not a suffix
    assert _fwd(levels=3, tiles=tiles(1, 1, T)) == U          # a single fused level
    assert _fwd(levels=4, tiles=tiles(T, T, T, T)) == U       # deeper than DWT2_TAIL_MAX
    assert _fwd(levels=3, tiles=tiles(1, -3, 1)) == U         # unknown negative id
    # accepted: the call goes on to the workspace check
    assert _fwd(levels=3, tiles=tiles(1, T, T)) == W
    assert _fwd(levels=3, tiles=tiles(T, T, T)) == W
    assert _lib.TAIL_MAX == 3
    import paper_1705_08266_amd as dwt
    assert dwt.fused_levels(4096, 4096, 5) == 3            # levels 3..5 (at most 3 fused)
    assert dwt.fused_levels(7680, 4320, 5) == 3            # levels 3..5 (1920x1080 and below)
    assert dwt.fused_levels(8192, 8192, 5) == 3            # levels 3..5 (2048^2 and below)
    assert dwt.fused_levels(16384, 16384, 5) == 2          # levels 4..5
    assert dwt.fused_levels(16384, 16384, 3) == 0          # level 3 alone is not fused
    assert dwt.fused_levels(512, 512, 1) == 0
    assert dwt.fused_levels(256, 384, 3) == 3
    assert _lib.load().dwt2_fused_levels(64, 64, 7) == _lib.ERR_INVALID_ARG


def test_exchange_ablation_scheme_limits():
    """The LDS-exchange schemes take FP32 only, and no fused levels or
    batches."""
    U, W = _lib.ERR_UNSUPPORTED, _lib.ERR_WORKSPACE
    for sch in (_lib.NONSEPARABLE_LDS, _lib.SEPARABLE_LDS):
        assert _fwd(levels=2, scheme=sch) == W                    # accepted up to the workspace
        assert _fwd(sd=_lib.Desc(64, 64, 64, _lib.F16), dd=_lib.Desc(64, 64, 64, _lib.F16),
                    scheme=sch) == U
        assert _fwd(levels=2, scheme=sch, tiles=(ctypes.c_int32 * 2)(_lib.TILE_TAIL,
                                                                      _lib.TILE_TAIL)) == U
        lib = _lib.load()
        img = (_lib.Image * 1)(_lib.Image(FAKE, 64, FAKE + (1 << 24), 64, None, 0, 64, 64))
        n = ctypes.c_size_t()
        assert lib.dwt2_batch_plan_bytes(img, 1, 0, 0, 1, 0, 0, None, 0, ctypes.byref(n)) == 0
        plan = (ctypes.c_ubyte * n.value)()
        assert lib.dwt2_batch_plan(img, 1, 0, 0, 1, 0, 0, None, 0, plan, n.value) == 0
        assert lib.dwt2_batch_run(plan, n.value, FAKE, sch, 0, None) == U
        assert lib.dwt2_forward_level_batch(None, 0, 0, sch, None, None) == U
    assert _fwd(scheme=4) == U


def test_inverse_argument_errors():
    lib = _lib.load()
    d = _lib.Desc(32, 32, 32, _lib.F32)
    assert lib.dwt2_inverse(None, ctypes.byref(d), FAKE, ctypes.byref(d), 0, 1, 0, 0,
                            None, 0, None) == _lib.ERR_INVALID_ARG
    assert lib.dwt2_inverse(FAKE, ctypes.byref(d), FAKE + 8, ctypes.byref(d), 0, 1, 0, 0,
                            None, 0, None) == _lib.ERR_INVALID_ARG
    assert lib.dwt2_inverse_ex(FAKE, ctypes.byref(d), FAKE + 8, ctypes.byref(d), 0, 1, 0, 0,
                               None, 0, None, None, None) == _lib.ERR_INVALID_ARG


def test_level_argument_errors():
    lib = _lib.load()
    B = FAKE + (1 << 30)
    # odd width
    assert lib.dwt2_forward_level(FAKE, 64, 0, 63, 64, B, 64, 0, B + 4096, B + 8192,
                                  B + 12288, 64, 0, 0, 0, -1, None) == _lib.ERR_INVALID_ARG
    # output overlaps input
    assert lib.dwt2_forward_level(FAKE, 64, 0, 64, 64, FAKE + 4, 64, 0, B, B + 8192,
                                  B + 16384, 64, 0, 0, 0, -1, None) == _lib.ERR_INVALID_ARG
    # tile id out of range
    assert lib.dwt2_forward_level(FAKE, 64, 0, 64, 64, B, 64, 0, B + 8192, B + 16384,
                                  B + 24576, 64, 0, 0, 0, 1000, None) == _lib.ERR_UNSUPPORTED
    # LL of a third dtype (F16 image, BF16 LL)
    assert lib.dwt2_inverse_level(B, 32, 2, B + 8192, B + 16384, B + 24576, 32, 1,
                                  FAKE, 64, 1, 64, 64, 0, 0, -1, None) == _lib.ERR_INVALID_ARG


def test_binding_refuses_cpu_tensors():
    torch = pytest.importorskip("torch")
    x = torch.zeros(8, 8)
    with pytest.raises(ValueError):
        dwt.forward(x)


def test_no_alloc_checks_before_touching_the_device():
    """dwt2_forward_no_alloc validates like dwt2_forward, then refuses sizes
    whose workspace exceeds its static array, all before any HIP call."""
    lib = _lib.load()
    big = _lib.Desc(16384, 16384, 16384, _lib.F32)
    assert lib.dwt2_forward_no_alloc(FAKE, ctypes.byref(big), FAKE + (1 << 32), ctypes.byref(big),
                                     0, 5, 0, 0, None) == _lib.ERR_WORKSPACE
    d = _lib.Desc(64, 64, 64, _lib.F32)
    assert lib.dwt2_forward_no_alloc(None, ctypes.byref(d), FAKE, ctypes.byref(d),
                                     0, 2, 0, 0, None) == _lib.ERR_INVALID_ARG
    assert lib.dwt2_forward_no_alloc(FAKE, ctypes.byref(d), FAKE + 8, ctypes.byref(d),
                                     0, 2, 0, 0, None) == _lib.ERR_INVALID_ARG   # overlap
    assert lib.dwt2_forward_no_alloc(FAKE, ctypes.byref(d), FAKE + (1 << 20), ctypes.byref(d),
                                     5, 2, 0, 0, None) == _lib.ERR_UNSUPPORTED
    assert _lib.STATIC_WORKSPACE_BYTES == 64 << 20
    header = open(HEADER).read()
    assert "#define DWT2_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)" in header


def test_head_tile_ids():
    """DWT2_TILE_HEAD marks exactly levels 1 and 2, with the tail (if any)
    starting at level 3 or later."""
    U, W, HD, T = _lib.ERR_UNSUPPORTED, _lib.ERR_WORKSPACE, _lib.TILE_HEAD, _lib.TILE_TAIL

    def tiles(*ids):
        return (ctypes.c_int32 * len(ids))(*ids)

    assert _fwd(levels=3, tiles=tiles(HD, HD, 0)) == W          # accepted up to the workspace
    assert _fwd(levels=5, tiles=tiles(HD, HD, T, T, T)) == W
    assert _fwd(levels=3, tiles=tiles(HD, 0, 0)) == U           # level 2 not marked
    assert _fwd(levels=3, tiles=tiles(0, HD, HD)) == U          # not levels 1 and 2
    assert _fwd(levels=1, tiles=tiles(HD)) == U                 # one level
    assert _fwd(levels=3, tiles=tiles(HD, HD, HD)) == U
    assert _fwd(levels=3, tiles=tiles(HD, T, T)) == U           # the tail would take level 2
    assert _fwd(levels=2, scheme=_lib.NONSEPARABLE_LDS, tiles=tiles(HD, HD)) == U
    assert dwt.head_levels(4096, 4096, 5) == 2                  # with the tail at levels 3..5
    assert dwt.head_levels(7680, 4320, 5) == 2
    assert dwt.head_levels(16384, 16384, 5) == 2
    assert dwt.head_levels(4096, 4096, 1) == 0
    assert dwt.head_levels(512, 512, 3) == 0                     # the tail takes every level
    assert _lib.load().dwt2_head_levels(64, 64, 7) == _lib.ERR_INVALID_ARG
