"""The exchange ablation: the same lifting with every neighbour exchange
through LDS and a barrier (horizontal ones included). Only where the
neighbour values come from changes, so results must be bit-identical to the
lane-shift kernels of the same scheme, for every 2-D tile configuration."""
import numpy as np
import pytest

import oracle
import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1705_08266_amd as dwt  # noqa: E402

PAIRS = [("nonseparable", "nonseparable_lds"), ("separable", "separable_lds")]


@pytest.mark.parametrize("wavelet", ["cdf97", "cdf53"])
@pytest.mark.parametrize("base,lds", PAIRS)
@pytest.mark.parametrize("shape,levels", [((512, 512), 5), ((264, 520), 3), ((2, 2), 1),
                                          ((130, 254), 1), ((136, 520), 3)])
def test_lds_exchange_equals_lane_shifts(wavelet, base, lds, shape, levels):
    x = torch.from_numpy(synthetic.uniform_image(*shape, seed=sum(shape))).to("cuda")
    tiles2d = [c[0] for c in dwt.tile_configs(wavelet)]
    ref_c = dwt.forward(x, wavelet, levels, base, tiles=[tiles2d[0]] * levels)
    ref_r = dwt.inverse(ref_c, wavelet, levels, base, tiles=[tiles2d[0]] * levels)
    for t in tiles2d:
        c = dwt.forward(x, wavelet, levels, lds, tiles=[t] * levels)
        r = dwt.inverse(ref_c, wavelet, levels, lds, tiles=[t] * levels)
        assert torch.equal(c, ref_c), (t, "forward")
        assert torch.equal(r, ref_r), (t, "inverse")


@pytest.mark.parametrize("lds", ["nonseparable_lds", "separable_lds"])
def test_lds_exchange_full_size_against_oracle(lds):
    x = synthetic.sinusoid_image(4096, 4096)
    xg = torch.from_numpy(x).to("cuda")
    c = dwt.forward(xg, "cdf97", 5, lds)
    assert torch.equal(c, dwt.forward(xg, "cdf97", 5, "nonseparable" if lds.startswith("non")
                                      else "separable", tiles=[0] * 5))
    ref = oracle.forward(x.astype(np.float64), "cdf97", 5, nthreads=16)
    assert np.abs(c.cpu().numpy() - ref).max() <= 1e-5 * 255
    r = dwt.inverse(c, "cdf97", 5, lds)
    assert (r - xg).abs().max().item() <= 1e-5 * 255
