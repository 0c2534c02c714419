"""Host-side arithmetic of bench.py, checked against closed forms: the
algorithmic bytes per direction of the one-pass-per-level method (read each
level's input once, write its four bands once), the bytes of the launches
actually made when the coarse levels are fused, the number of rotating buffer
sets, and the one-GPU guard. No GPU is touched."""
import importlib.util
import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("levels", [1, 2, 3, 5, 6])
def test_fp32_bytes_per_pixel_closed_form(bench, levels):
    # FP32 everywhere: level j moves 8 bytes per input pixel, and its input
    # has 4^-(j-1) of the image's pixels
    W = H = 4096
    per_px = sum(bench.level_bytes(W, H, levels, 4)) / (W * H)
    assert per_px == pytest.approx(8 * sum(4.0 ** -j for j in range(levels)), rel=0, abs=1e-12)


def test_fp32_five_levels_figures(bench):
    W = H = 4096
    lb = bench.level_bytes(W, H, 5, 4)
    assert lb[0] == 134217728                      # 64 MiB read + 64 MiB of bands written
    assert 2 * sum(lb) / (W * H) == 21.3125        # forward + inverse


def test_fp16_with_fp32_intermediates(bench):
    # level 1: 2 (read) + 1.5 (three 16-bit bands) + 1 (FP32 low-low);
    # middle levels: 4 + 1.5 + 1; the last level: 4 + 1.5 + 0.5 (16-bit LL)
    W = H = 4096
    per_px = sum(bench.level_bytes(W, H, 5, 2)) / (W * H)
    want = 4.5 + 6.5 / 4 + 6.5 / 16 + 6.5 / 64 + 6.0 / 256
    assert per_px == pytest.approx(want, rel=0, abs=1e-12)
    assert want == 6.65625


def test_executed_bytes_with_fused_tail(bench):
    W = H = 4096
    lb = bench.level_bytes(W, H, 5, 4)
    # without fusion the executed bytes are the per-level bytes
    assert bench.executed_bytes(W, H, 5, 4, 0) == sum(lb)
    assert bench.executed_bytes(W, H, 5, 4, 1) == sum(lb)
    # levels 3..5 fused: read the level-3 input (1024^2 FP32) once, write the
    # detail bands of levels 3, 4, 5 and the final LL once
    tail = 1024 * 1024 * 4 + 3 * 4 * (512 * 512 + 256 * 256 + 128 * 128) + 128 * 128 * 4
    assert tail == 8388608
    assert bench.executed_bytes(W, H, 5, 4, 3) == lb[0] + lb[1] + tail
    assert 2 * bench.executed_bytes(W, H, 5, 4, 3) / (W * H) == 21.0
    # the saving equals the intermediate low-low bands written and re-read
    saved = sum(lb) - bench.executed_bytes(W, H, 5, 4, 3)
    assert saved == 2 * 4 * (512 * 512 + 256 * 256)


@pytest.mark.parametrize("dtype,W,H,want", [
    ("f32", 4096, 4096, 8), ("f16", 4096, 4096, 16), ("f32", 2048, 2048, 32),
    ("f32", 16384, 16384, 4), ("f32", 7680, 4320, 5), ("f32", 512, 512, 64)])
def test_buffer_sets_exceed_twice_the_cache(bench, dtype, W, H, want):
    args = types.SimpleNamespace(sets=None, dtype=dtype)
    n = bench.buffer_sets(args, W, H)
    assert n == want
    es = {"f32": 4, "f16": 2}[dtype]
    if 4 < n < 64:
        assert n * W * H * es >= 2 * bench.INFINITY_CACHE_BYTES > (n - 1) * W * H * es
    assert bench.buffer_sets(types.SimpleNamespace(sets=3, dtype=dtype), W, H) == 3


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=120,
                       env={**os.environ, "WORLD_SIZE": "1"})
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_launch_units_of_the_chain(bench):
    assert bench.launch_units(5, 3, True) == [("head", 1, 2), ("tail", 3, 3)]
    assert bench.launch_units(5, 2, True) == [("head", 1, 2), ("level", 3, 1), ("tail", 4, 2)]
    assert bench.launch_units(5, 0, True) == [("head", 1, 2), ("level", 3, 1), ("level", 4, 1),
                                              ("level", 5, 1)]
    assert bench.launch_units(3, 3, False) == [("tail", 1, 3)]
    assert bench.launch_units(2, 0, False) == [("level", 1, 1), ("level", 2, 1)]


def test_executed_bytes_with_fused_head(bench):
    W = H = 4096
    lb = bench.level_bytes(W, H, 5, 4)
    head = bench.unit_bytes(W, H, 5, 4, ("head", 1, 2))
    # read the image once, write the detail bands of levels 1 and 2 and the
    # level-2 LL (FP32) once: 8 bytes per image pixel, as level 1 alone
    assert head == W * H * 4 + 3 * 4 * (2048 * 2048 + 1024 * 1024) + 1024 * 1024 * 4
    assert head == lb[0] == 134217728
    # the saving is the level-1 LL written and read back
    assert lb[0] + lb[1] - head == 2 * 4 * 2048 * 2048
    tail = bench.unit_bytes(W, H, 5, 4, ("tail", 3, 3))
    assert tail == 8388608
    assert bench.executed_bytes(W, H, 5, 4, 3, head=True) == head + tail
    assert 2 * bench.executed_bytes(W, H, 5, 4, 3, head=True) / (W * H) == 17.0
    # a single-level unit is the per-level method's level
    for j in range(1, 6):
        assert bench.unit_bytes(W, H, 5, 4, ("level", j, 1)) == lb[j - 1]
    # FP16 storage: the head writes 16-bit bands and an FP32 level-2 LL
    lb16 = bench.level_bytes(W, H, 5, 2)
    assert bench.unit_bytes(W, H, 5, 2, ("head", 1, 2)) == lb16[0] + lb16[1] - 2 * 4 * 2048 * 2048


def test_ab_workload_needs_the_other_build():
    """The two-build comparison refuses to run without the second library,
    before touching a GPU."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "ab"],
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=120,
                       cwd=ROOT)
    assert r.returncode == 2
    assert "--other-lib" in r.stderr
    assert r.stdout == ""
