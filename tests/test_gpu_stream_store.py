"""Non-temporal output of the multi-level inverse: when the reconstructed image
holds 32 MiB to 256 MiB, the finest level of dwt2_inverse writes it with
non-temporal stores. The values must be bit-identical to the one-level entry
point, which always writes through the caches, for every storage type and
scheme, on images at, just inside and just outside both size limits, with
pitched and unpitched outputs."""
import pytest

import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1705_08266_amd as dwt  # noqa: E402

TDT = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}
ES = {"f32": 4, "f16": 2, "bf16": 2}
LIMITS = (32 << 20, 256 << 20)

# (height, width, storage): FP32 4096^2 and FP16 8192x4096 are 64 MiB, FP16
# 4096^2 exactly 32 MiB, FP32 4096x2040 just below it; FP32 8192^2 exactly
# 256 MiB, FP32 8192x8200 just above it
CASES = [((4096, 4096), "f32"), ((4096, 8192), "f16"), ((4096, 4096), "bf16"),
         ((4096, 4096), "f16"), ((2040, 4096), "f32"), ((4094, 4100), "f32"),
         ((8192, 8192), "f32"), ((8192, 8200), "f32")]


def _inverse_one_level_reference(c, wavelet, scheme, out):
    h, w = c.shape
    dwt.inverse_level(c[:h // 2, :w // 2], c[:h // 2, w // 2:], c[h // 2:, :w // 2],
                      c[h // 2:, w // 2:], out, wavelet, scheme)
    return out


@pytest.mark.parametrize("scheme", ["nonseparable", "separable"])
@pytest.mark.parametrize("shape,dtype", CASES)
def test_streamed_output_equals_cached(shape, dtype, scheme):
    h, w = shape
    streamed = LIMITS[0] <= h * w * ES[dtype] <= LIMITS[1]
    print(f"stream {dtype} {shape} {scheme} streamed={streamed}", flush=True)
    x = torch.from_numpy(synthetic.uniform_image(h, w, seed=h + w)).to("cuda").to(TDT[dtype])
    c = dwt.forward(x, "cdf97", 1, scheme)
    got = dwt.inverse(c, "cdf97", 1, scheme)
    want = _inverse_one_level_reference(c, "cdf97", scheme, torch.empty_like(c))
    assert torch.equal(got, want)


@pytest.mark.parametrize("levels", [2, 5])
def test_streamed_multilevel_equals_per_level(levels):
    """Five levels at 4096^2 FP32: the fused tail and level 2 write the
    workspace, level 1 streams the image; the per-level chain matches bit for
    bit."""
    h = w = 4096
    print(f"stream multilevel L={levels}", flush=True)
    x = torch.from_numpy(synthetic.uniform_image(h, w, seed=7)).to("cuda")
    c = dwt.forward(x, "cdf97", levels)
    got = dwt.inverse(c, "cdf97", levels)
    cur = c[:h >> levels, :w >> levels].clone()   # the coarsest low-low band
    for j in range(levels, 0, -1):
        hh, ww = h >> (j - 1), w >> (j - 1)
        out = torch.empty(hh, ww, device="cuda")
        blk = c[:hh, :ww].clone()
        blk[:hh // 2, :ww // 2] = cur
        cur = _inverse_one_level_reference(blk, "cdf97", "nonseparable", out)
    assert torch.equal(got, cur)


def test_streamed_pitched_output():
    """A destination view inside a wider buffer (pitch > width): aligned
    pitches take the vector (streamed) stores, an odd pitch the per-element
    ones; both equal the unpitched result."""
    h, w = 4096, 4096
    print("stream pitched", flush=True)
    x = torch.from_numpy(synthetic.uniform_image(h, w, seed=11)).to("cuda")
    c = dwt.forward(x, "cdf97", 3)
    want = dwt.inverse(c, "cdf97", 3)
    for pitch in (w + 64, w + 1):
        big = torch.full((h, pitch), float("nan"), device="cuda")
        got = dwt.inverse(c, "cdf97", 3, out=big[:, :w])
        assert torch.equal(got, want)
        assert torch.isnan(big[:, w:]).all()
