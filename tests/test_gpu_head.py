"""Fused finest levels (levels 1 and 2 in one launch, the band between them
in LDS): bit-identical to one launch per level for every wavelet, scheme and
storage type, on shapes that put the image edges inside one window, ragged
block counts along each axis and windows wider than the image; together
with the fused tail; and within the FP32 bound of the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1705_08266_amd as dwt  # noqa: E402
from paper_1705_08266_amd import _lib  # noqa: E402

HD, T = _lib.TILE_HEAD, _lib.TILE_TAIL
TDT = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}

# (height, width), levels. The forward head owns 116-quad wide blocks of
# level 1 (58 of level 2) and 36 quad rows of level 1; the inverse owns
# 116 x 44 level-1 quads: the shapes below are single-block, exact-multiple
# and ragged along each axis.
SHAPES = [((8, 8), 2), ((64, 64), 2), ((96, 232), 2), ((144, 464), 2), ((148, 468), 2),
          ((176, 464), 3), ((1000, 1004), 2), ((1024, 1024), 3), ((4, 2048), 2),
          ((2048, 12), 2), ((1088, 1920), 4)]


def _per_level(levels):
    return [0] * levels


def _head(levels):
    return [HD, HD] + [0] * (levels - 2)


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("wavelet", ["cdf97", "cdf53"])
@pytest.mark.parametrize("scheme", ["nonseparable", "separable"])
@pytest.mark.parametrize("shape,levels", SHAPES)
def test_head_equals_per_level(dtype, wavelet, scheme, shape, levels):
    print(f"head {dtype} {wavelet} {scheme} {shape} L={levels}", flush=True)
    x = torch.from_numpy(synthetic.uniform_image(*shape, seed=sum(shape) + levels))
    x = x.to("cuda").to(TDT[dtype])
    per = dwt.forward(x, wavelet, levels, scheme, tiles=_per_level(levels))
    fus = dwt.forward(x, wavelet, levels, scheme, tiles=_head(levels))
    torch.cuda.synchronize()
    assert torch.equal(per, fus)
    rp = dwt.inverse(per, wavelet, levels, scheme, tiles=_per_level(levels))
    rf = dwt.inverse(per, wavelet, levels, scheme, tiles=_head(levels))
    torch.cuda.synchronize()
    assert torch.equal(rp, rf)


@pytest.mark.parametrize("wavelet", ["cdf97", "cdf53"])
@pytest.mark.parametrize("shape,levels,fused", [((512, 512), 5, 3), ((1056, 2016), 5, 2),
                                                ((256, 384), 5, 3)])
def test_head_with_tail_equals_per_level(wavelet, shape, levels, fused):
    x = torch.from_numpy(synthetic.uniform_image(*shape, seed=7)).to("cuda")
    tiles = [HD, HD] + [0] * (levels - 2 - fused) + [T] * fused
    per = dwt.forward(x, wavelet, levels, tiles=_per_level(levels))
    fus = dwt.forward(x, wavelet, levels, tiles=tiles)
    assert torch.equal(per, fus)
    assert torch.equal(dwt.inverse(per, wavelet, levels, tiles=_per_level(levels)),
                       dwt.inverse(per, wavelet, levels, tiles=tiles))


@pytest.mark.parametrize("wavelet", ["cdf97", "cdf53"])
@pytest.mark.parametrize("shape,levels", [((148, 468), 2), ((1000, 1008), 3), ((64, 64), 2)])
def test_head_against_oracle(wavelet, shape, levels):
    x = synthetic.uniform_image(*shape, seed=5)
    xg = torch.from_numpy(x).to("cuda")
    c = dwt.forward(xg, wavelet, levels, tiles=_head(levels))
    ref = oracle.forward(x.astype(np.float64), wavelet, levels)
    assert np.abs(c.cpu().numpy() - ref).max() <= 1e-5 * 255
    refc = ref.astype(np.float32)
    r = dwt.inverse(torch.from_numpy(refc).to("cuda"), wavelet, levels, tiles=_head(levels))
    ref_r = oracle.inverse(refc.astype(np.float64), wavelet, levels)
    assert np.abs(r.cpu().numpy() - ref_r).max() <= 1e-5 * 255


def test_default_uses_the_head_at_the_headline_size():
    assert dwt.head_levels(4096, 4096, 5) == 2
    x = torch.from_numpy(synthetic.sinusoid_image(4096, 4096)).to("cuda")
    c = dwt.forward(x, "cdf97", 5)
    per = dwt.forward(x, "cdf97", 5, tiles=_per_level(5))
    assert torch.equal(c, per)
    r = dwt.inverse(c, "cdf97", 5)
    assert torch.equal(r, dwt.inverse(c, "cdf97", 5, tiles=_per_level(5)))
    assert (r - x).abs().max().item() <= 1e-5 * 255
