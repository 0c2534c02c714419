"""Seeded random shapes against the FP64 oracle: widths and heights that are
multiples of 2^L but not of the tile sizes, all level counts whose coarsest
level is at least 2x2, both wavelets and both schemes, default launches
(which fuse the small trailing levels) and one launch per level. FP32 bound:
1e-5 of max|x| for the forward coefficients, the inverse of the oracle's
coefficients, and the round trip."""
import numpy as np
import pytest

import oracle
import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1705_08266_amd as dwt  # noqa: E402


def _cases(n=24, seed=20240601):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        L = int(rng.integers(1, 7))
        m = 1 << L
        w = int(rng.integers(1, max(2, 1400 // m))) * m
        h = int(rng.integers(1, max(2, 1400 // m))) * m
        if (w >> L) < 1 or (h >> L) < 1 or w < 2 or h < 2:
            continue
        out.append((h, w, L, str(rng.choice(["cdf97", "cdf53"])),
                    str(rng.choice(["nonseparable", "separable"]))))
    return out


@pytest.mark.parametrize("h,w,levels,wavelet,scheme", _cases())
def test_random_shape_against_oracle(h, w, levels, wavelet, scheme):
    print(f"random {h}x{w} L={levels} {wavelet} {scheme} fused={dwt.fused_levels(w, h, levels)}",
          flush=True)
    x = synthetic.uniform_image(h, w, seed=h * 7919 + w)
    x64 = x.astype(np.float64)
    xg = torch.from_numpy(x).to("cuda")
    ref = oracle.forward(x64, wavelet, levels)
    c = dwt.forward(xg, wavelet, levels, scheme)
    c1 = dwt.forward(xg, wavelet, levels, scheme, tiles=[dwt.default_tile(w, h)] * levels)
    assert torch.equal(c, c1)
    assert np.abs(c.cpu().numpy() - ref).max() <= 1e-5 * 255
    ref32 = ref.astype(np.float32)
    r = dwt.inverse(torch.from_numpy(ref32).to("cuda"), wavelet, levels, scheme)
    ref_r = oracle.inverse(ref32.astype(np.float64), wavelet, levels)
    assert np.abs(r.cpu().numpy() - ref_r).max() <= 1e-5 * 255
    rt = dwt.inverse(c, wavelet, levels, scheme)
    assert np.abs(rt.cpu().numpy() - x64).max() <= 1e-5 * 255
