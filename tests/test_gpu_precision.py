"""FP16 and BF16 storage with FP32 lifting arithmetic, against the FP64 oracle.

The image and the coefficient buffers are 16-bit; intermediate low-low bands
between levels stay FP32 (the library's workspace). Errors are relative to
max|x| and measured per result:
  forward     GPU coefficients vs the oracle forward of the same stored image
  inverse     GPU inverse of the oracle coefficients rounded to the storage
              type vs the oracle inverse of those same rounded coefficients
  round trip  GPU inverse of GPU coefficients vs the stored image
Stated bounds (rounding to nearest even at every store):
  FP16: 1e-3 forward and inverse, 2e-3 round trip;
  BF16: 5e-3 forward and inverse, 1e-2 round trip (8-bit significand).
For 0..255 images the forward error is one rounding of each coefficient, at
most half an FP16 ulp of the largest one (0.0625 at 255: 2.45e-4 of max|x|,
which the 16384^2 forward reaches). The round trip adds the inverse's
amplification of those roundings through five levels of synthesis filters
and the final rounding of the image (9.8e-4 measured at 16384^2); its bound
is the 2e-3 cap that FP16 storage is held to, twice the largest measured
value. The inverse alone (one set of rounded coefficients in, one rounding
out) stays below 1e-3.
"""
import numpy as np
import pytest

import oracle
import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1705_08266_amd as dwt  # noqa: E402

BOUNDS = {
    "f16": dict(forward=1e-3, inverse=1e-3, round_trip=2e-3),
    "bf16": dict(forward=5e-3, inverse=5e-3, round_trip=1e-2),
}
TDT = {"f16": torch.float16, "bf16": torch.bfloat16}


def _errors(x_stored, dtype, wavelet, levels, scheme="nonseparable", nthreads=8):
    t = TDT[dtype]
    x64 = x_stored.astype(np.float64)
    scale = float(np.abs(x64).max())
    xg = torch.from_numpy(x_stored).to("cuda").to(t)
    c = dwt.forward(xg, wavelet, levels, scheme)
    ref_c = oracle.forward(x64, wavelet, levels, nthreads=nthreads)
    c_h = c.float().cpu().numpy().astype(np.float64)
    e_fwd = np.abs(c_h - ref_c).max() / scale
    # inverse of the oracle's coefficients, rounded to the storage type
    c_in = torch.from_numpy(ref_c.astype(np.float32)).to("cuda").to(t)
    c_in64 = c_in.float().cpu().numpy().astype(np.float64)
    r = dwt.inverse(c_in, wavelet, levels, scheme)
    ref_r = oracle.inverse(c_in64, wavelet, levels, nthreads=nthreads)
    e_inv = np.abs(r.float().cpu().numpy() - ref_r).max() / scale
    rt = dwt.inverse(c, wavelet, levels, scheme)
    e_rt = np.abs(rt.float().cpu().numpy() - x64).max() / scale
    torch.cuda.synchronize()
    return dict(forward=float(e_fwd), inverse=float(e_inv), round_trip=float(e_rt))


def _check(errs, dtype):
    for k, v in errs.items():
        assert v <= BOUNDS[dtype][k], (dtype, k, v, errs)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
@pytest.mark.parametrize("wavelet", ["cdf97", "cdf53"])
@pytest.mark.parametrize("scheme", ["nonseparable", "separable"])
@pytest.mark.parametrize("shape,levels", [((512, 512), 5), ((264, 520), 3), ((2, 2), 1),
                                          ((130, 254), 1)])
def test_storage_precision_small(dtype, wavelet, scheme, shape, levels):
    x = synthetic.uniform_image(*shape, seed=17 + levels)   # 0..255 is exact in both types
    errs = _errors(x, dtype, wavelet, levels, scheme)
    print(f"{dtype} {wavelet} {scheme} {shape} L={levels}: {errs}", flush=True)
    _check(errs, dtype)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_every_tile_config_matches_in_16_bit(dtype):
    x = torch.from_numpy(synthetic.uniform_image(136, 520, seed=3)).to("cuda").to(TDT[dtype])
    outs = []
    for t in range(len(dwt.tile_configs("cdf97"))):
        c = dwt.forward(x, "cdf97", 3, tiles=[t] * 3)
        r = dwt.inverse(c, "cdf97", 3, tiles=[t] * 3)
        outs.append((c.float().cpu().numpy(), r.float().cpu().numpy()))
    for t in range(1, len(outs)):
        assert np.array_equal(outs[0][0], outs[t][0]), t
        assert np.array_equal(outs[0][1], outs[t][1]), t


def test_fp16_7680x4320_five_levels():
    """The bandwidth-sweep workload stored as FP16 (uniform integers)."""
    x = synthetic.uniform_image(4320, 7680, seed=synthetic.SEED_BASE + 3)
    errs = _errors(x, "f16", "cdf97", 5, nthreads=16)
    print(f"f16 7680x4320 L=5: {errs}", flush=True)
    _check(errs, "f16")


def test_fp16_16384_five_levels():
    """The largest bandwidth-sweep workload stored as FP16, whole arrays
    against the oracle."""
    x = synthetic.uniform_image(16384, 16384, seed=synthetic.SEED_BASE + 3)
    errs = _errors(x, "f16", "cdf97", 5, nthreads=16)
    print(f"f16 16384^2 L=5: {errs}", flush=True)
    _check(errs, "f16")


def test_fp32_16384_five_levels():
    """The largest bandwidth-sweep workload in FP32: forward against the
    oracle, the inverse of the oracle's coefficients against the oracle's
    inverse of the same (FP32-rounded) coefficients, and the round trip."""
    x = synthetic.uniform_image(16384, 16384, seed=synthetic.SEED_BASE + 3)
    x64 = x.astype(np.float64)
    xg = torch.from_numpy(x).to("cuda")
    c = dwt.forward(xg, "cdf97", 5)
    ref = oracle.forward(x64, "cdf97", 5, nthreads=16)
    e_fwd = np.abs(c.cpu().numpy() - ref).max() / 255.0
    del x64
    ref32 = ref.astype(np.float32)
    del ref
    r = dwt.inverse(torch.from_numpy(ref32).to("cuda"), "cdf97", 5)
    ref_r = oracle.inverse(ref32.astype(np.float64), "cdf97", 5, nthreads=16)
    e_inv = np.abs(r.cpu().numpy() - ref_r).max() / 255.0
    del ref_r, r
    rt = dwt.inverse(c, "cdf97", 5)
    e_rt = np.abs(rt.cpu().numpy() - x).max() / 255.0
    print(f"f32 16384^2 L=5: fwd {e_fwd:.3e} inv {e_inv:.3e} rt {e_rt:.3e}", flush=True)
    assert e_fwd <= 1e-5 and e_inv <= 1e-5 and e_rt <= 1e-5
