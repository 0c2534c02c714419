"""Parity of the HIP path with the FP64 oracle, through the C ABI, on MI355X.

Tolerance for FP32 storage and FP32 arithmetic: max |gpu - oracle| <= 1e-5 *
max|x| for the forward coefficients, the inverse of oracle coefficients, and
the round trip.
"""
import numpy as np
import pytest

import oracle
import synthetic

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_1705_08266_amd as dwt  # noqa: E402

TOL32 = 1e-5
SCHEMES = ["nonseparable", "separable"]
WAVELETS = ["cdf97", "cdf53"]


def _gpu(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda").to(dtype)


def _host(t):
    torch.cuda.synchronize()
    return t.float().cpu().numpy().astype(np.float64)


def _rel(a, b, scale):
    return float(np.max(np.abs(a - b)) / scale) if a.size else 0.0


def _check_all(x32, wavelet, levels, scheme, tiles=None):
    """Forward, inverse-of-oracle and round trip against the oracle."""
    x = x32.astype(np.float64)
    scale = max(1.0, float(np.max(np.abs(x))))
    ref_c = oracle.forward(x, wavelet, levels, nthreads=8)
    xg = _gpu(x32)
    c = dwt.forward(xg, wavelet, levels, scheme, tiles=tiles)
    e_fwd = _rel(_host(c), ref_c, scale)
    c_in = _gpu(ref_c.astype(np.float32))
    r = dwt.inverse(c_in, wavelet, levels, scheme, tiles=tiles)
    ref_r = oracle.inverse(ref_c.astype(np.float32).astype(np.float64), wavelet, levels,
                           nthreads=8)
    e_inv = _rel(_host(r), ref_r, scale)
    rt = dwt.inverse(c, wavelet, levels, scheme, tiles=tiles)
    e_rt = _rel(_host(rt), x, scale)
    return e_fwd, e_inv, e_rt


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("wavelet", WAVELETS)
def test_small_image_one_level(wavelet, scheme):
    x = synthetic.uniform_image(512, 512)
    print(f"case 512x512 {wavelet} {scheme} L=1", flush=True)
    e = _check_all(x, wavelet, 1, scheme)
    assert max(e) <= TOL32, e


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("wavelet", WAVELETS)
@pytest.mark.parametrize("shape,levels", [((264, 520), 3), ((130, 254), 1),
                                          ((96, 1000), 3), ((1000, 96), 3),
                                          ((64, 64), 6), ((2, 2), 1), ((4, 6), 1),
                                          ((6, 4), 1), ((2, 512), 1), ((512, 2), 1),
                                          ((40, 24), 3)])
def test_ragged_and_tiny_shapes(wavelet, scheme, shape, levels):
    x = synthetic.uniform_image(*shape, seed=sum(shape) + levels)
    print(f"case {shape} {wavelet} {scheme} L={levels}", flush=True)
    e = _check_all(x, wavelet, levels, scheme)
    assert max(e) <= TOL32, e


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("wavelet", WAVELETS)
def test_every_tile_config_gives_identical_bits(wavelet, scheme):
    """Each output quad goes through the same FMAs whatever the tile shape, so
    all tile configurations must agree bit for bit; a halo or barrier bug
    shows up as a difference."""
    x = _gpu(synthetic.uniform_image(200, 744, seed=11))
    ntiles = len(dwt.tile_configs(wavelet))
    outs, invs = [], []
    for t in range(ntiles):
        print(f"case tile {t} {wavelet} {scheme}", flush=True)
        c = dwt.forward(x, wavelet, 2, scheme, tiles=[t, t])
        outs.append(_host(c))
        invs.append(_host(dwt.inverse(c, wavelet, 2, scheme, tiles=[t, t])))
    for t in range(1, ntiles):
        assert np.array_equal(outs[0], outs[t]), t
        assert np.array_equal(invs[0], invs[t]), t


def test_nonseparable_and_separable_agree():
    x = _gpu(synthetic.sinusoid_image(512, 768, seed=3))
    a = _host(dwt.forward(x, "cdf97", 4, "nonseparable"))
    b = _host(dwt.forward(x, "cdf97", 4, "separable"))
    assert np.max(np.abs(a - b)) <= TOL32 * 255


def test_pitched_views_and_level_entry_points():
    """Buffers with a pitch larger than the width (views into a wider array)."""
    x_full = synthetic.uniform_image(128, 300, seed=5)
    big = _gpu(x_full)
    xv = big[:, 20:276]                      # 128 x 256 view, pitch 300
    outbig = torch.zeros(128, 260, device="cuda")
    cv = outbig[:, 2:258]                    # pitch 260
    dwt.forward(xv, "cdf97", 3, out=cv)
    ref = oracle.forward(x_full[:, 20:276].astype(np.float64), "cdf97", 3)
    assert _rel(_host(cv), ref, 255) <= TOL32
    assert np.all(_host(outbig[:, :2]) == 0) and np.all(_host(outbig[:, 258:]) == 0)
    # single level through dwt2_forward_level into separate band tensors
    xs = _gpu(x_full[:, :256])
    bands = [torch.empty(64, 128, device="cuda") for _ in range(4)]
    mall = torch.empty(128, 256, device="cuda")
    hl, lh, hh = mall[:64, 128:], mall[64:, :128], mall[64:, 128:]
    dwt.forward_level(xs, bands[0], hl, lh, hh, "cdf53")
    ref1 = oracle.forward(x_full[:, :256].astype(np.float64), "cdf53", 1)
    got = _host(mall)
    got[:64, :128] = _host(bands[0])
    assert _rel(got, ref1, 255) <= TOL32
    rec = torch.empty(128, 256, device="cuda")
    dwt.inverse_level(bands[0], hl, lh, hh, rec, "cdf53")
    assert _rel(_host(rec), x_full[:, :256].astype(np.float64), 255) <= TOL32


def test_constant_image_exact_structure():
    x = _gpu(np.full((256, 512), 100.0, dtype=np.float32))
    c = _host(dwt.forward(x, "cdf97", 5))
    ll = c[:8, :16]
    assert np.max(np.abs(ll - 100.0)) <= 1e-4
    c[:8, :16] = 0
    assert np.max(np.abs(c)) <= 1e-4


def test_invalid_arguments_raise():
    x = torch.zeros(48, 64, device="cuda")
    with pytest.raises(dwt.DWT2Error):
        dwt.forward(x, "cdf97", 5)           # 48 not divisible by 32
    with pytest.raises(dwt.DWT2Error):
        dwt.forward(x, "cdf97", 1, out=x)    # in place is refused


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("wavelet", WAVELETS)
@pytest.mark.parametrize("levels", [1, 5])
def test_full_size_4096_sinusoids(wavelet, scheme, levels):
    """The benchmark workload at full size, default tiles (the bench's launch
    configuration), whole arrays against the oracle."""
    x = synthetic.sinusoid_image(4096, 4096)
    print(f"case 4096^2 {wavelet} {scheme} L={levels}", flush=True)
    e = _check_all(x, wavelet, levels, scheme)
    print(f"errors fwd/inv/rt {e}", flush=True)
    assert max(e) <= TOL32, e


def test_full_size_7680x4320():
    x = synthetic.uniform_image(4320, 7680, seed=synthetic.SEED_BASE + 3)
    print("case 7680x4320 cdf97 L=5", flush=True)
    e = _check_all(x, "cdf97", 5, "nonseparable")
    print(f"errors fwd/inv/rt {e}", flush=True)
    assert max(e) <= TOL32, e
