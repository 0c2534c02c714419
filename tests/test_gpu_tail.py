"""Fused coarse levels (one launch for the last 2..3 levels): bit-identical to
running the same levels one launch each, for every wavelet, scheme and
storage type, on shapes that put the fused region's edges, the image edges
and ragged block counts in every combination; and within the FP32 bound of
the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1705_08266_amd as dwt  # noqa: E402
from paper_1705_08266_amd import _lib  # noqa: E402

T = _lib.TILE_TAIL
TDT = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}

# (height, width, levels, fused levels)
SHAPES = [((512, 512), 5, 3), ((520, 264), 3, 3), ((384, 256), 3, 2), ((2032, 1040), 3, 2),
          ((96, 64), 2, 2), ((4, 4), 2, 2), ((8, 8), 3, 3), ((520, 136), 3, 3),
          ((2048, 32), 4, 3), ((8, 4096), 3, 3), ((1216, 192), 6, 3), ((4320 // 4, 7680 // 4), 3, 2)]


def _tiles(levels, fused):
    return [1] * (levels - fused) + [T] * fused


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("wavelet", ["cdf97", "cdf53"])
@pytest.mark.parametrize("scheme", ["nonseparable", "separable"])
@pytest.mark.parametrize("shape,levels,fused", SHAPES)
def test_fused_tail_equals_per_level(dtype, wavelet, scheme, shape, levels, fused):
    print(f"tail {dtype} {wavelet} {scheme} {shape} L={levels} F={fused}", flush=True)
    x = torch.from_numpy(synthetic.uniform_image(*shape, seed=sum(shape) + levels))
    x = x.to("cuda").to(TDT[dtype])
    per = dwt.forward(x, wavelet, levels, scheme, tiles=[1] * levels)
    fus = dwt.forward(x, wavelet, levels, scheme, tiles=_tiles(levels, fused))
    assert torch.equal(per, fus)
    rp = dwt.inverse(per, wavelet, levels, scheme, tiles=[1] * levels)
    rf = dwt.inverse(per, wavelet, levels, scheme, tiles=_tiles(levels, fused))
    assert torch.equal(rp, rf)


@pytest.mark.parametrize("wavelet", ["cdf97", "cdf53"])
@pytest.mark.parametrize("shape,levels,fused", SHAPES[:6])
def test_fused_tail_against_oracle(wavelet, shape, levels, fused):
    x = synthetic.uniform_image(*shape, seed=3)
    x64 = x.astype(np.float64)
    xg = torch.from_numpy(x).to("cuda")
    c = dwt.forward(xg, wavelet, levels, tiles=_tiles(levels, fused))
    ref = oracle.forward(x64, wavelet, levels)
    assert np.abs(c.cpu().numpy() - ref).max() <= 1e-5 * 255
    r = dwt.inverse(torch.from_numpy(ref.astype(np.float32)).to("cuda"), wavelet, levels,
                    tiles=_tiles(levels, fused))
    ref_r = oracle.inverse(ref.astype(np.float32).astype(np.float64), wavelet, levels)
    assert np.abs(r.cpu().numpy() - ref_r).max() <= 1e-5 * 255


@pytest.mark.parametrize("shape", [(4096, 4096), (4320, 7680)])
def test_default_fusion_at_full_size_equals_per_level(shape):
    """The library fuses the levels whose input has at most 2^20 pixels by
    default (4096^2, 5 levels: levels 3-5; 7680x4320: levels 4-5)."""
    x = torch.from_numpy(synthetic.sinusoid_image(*shape)).to("cuda")
    for wavelet in ("cdf97", "cdf53"):
        c_def = dwt.forward(x, wavelet, 5)
        c_per = dwt.forward(x, wavelet, 5, tiles=[1] * 5)
        assert torch.equal(c_def, c_per)
        r_def = dwt.inverse(c_def, wavelet, 5)
        r_per = dwt.inverse(c_def, wavelet, 5, tiles=[1] * 5)
        assert torch.equal(r_def, r_per)
        assert (r_def - x).abs().max().item() <= 1e-5 * 255


def test_fused_tail_in_a_captured_graph():
    x = torch.from_numpy(synthetic.uniform_image(512, 512, seed=8)).to("cuda")
    out = torch.empty_like(x)
    back = torch.empty_like(x)
    ws = dwt.make_workspace(512, 512, 5)
    dwt.forward(x, "cdf97", 5, out=out, workspace=ws)
    dwt.inverse(out, "cdf97", 5, out=back, workspace=ws)
    torch.cuda.synchronize()
    ref_c, ref_r = out.clone(), back.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        dwt.forward(x, "cdf97", 5, out=out, workspace=ws)
        dwt.inverse(out, "cdf97", 5, out=back, workspace=ws)
    for k in range(3):
        out.zero_()
        back.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref_c) and torch.equal(back, ref_r), k


def test_level_events_bracket_the_fused_launch():
    x = torch.from_numpy(synthetic.uniform_image(512, 512, seed=1)).to("cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(10)]
    dwt.forward(x, "cdf97", 5, events=ev)
    torch.cuda.synchronize()
    ms = [ev[2 * j].elapsed_time(ev[2 * j + 1]) for j in range(5)]
    assert ms[2] > 0 and all(m >= 0 for m in ms)
    assert ms[3] <= ms[2] and ms[4] <= ms[2]
