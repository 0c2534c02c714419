"""Closed-form CDF filters and a direct-convolution 2-D filter bank (FP64).

TEST INFRASTRUCTURE (part of the oracle): used only to pin the lifting oracle.

The paper writes the transform as a pair of FIR filters G0, G1 followed by
subsampling by two (Sec. 2, eq. 1) and factors that filter bank into lifting
steps (eq. 2). It cites the CDF wavelets without printing their taps, so the
taps are derived here from first principles, independently of any lifting
constant:

  * Let y = sin^2(w/2) = (2 - z - 1/z)/4 and c = cos^2(w/2) = (2 + z + 1/z)/4.
    The Daubechies product filter of order N is c^N * P_N(y) with
    P_N(y) = sum_{k<N} C(N-1+k, k) y^k.
  * CDF 5/3 (N = 2): analysis low-pass c * (1 + 2y), synthesis low-pass c.
  * CDF 9/7 (N = 4): P_4(y) = 1 + 4y + 10y^2 + 20y^3 has one real root y_r.
    Synthesis low-pass c^2 * (1 - y/y_r) (7 taps); analysis low-pass
    c^2 * P_4(y) / (1 - y/y_r) (9 taps).
  * Both low-pass filters have DC gain 1. The analysis high-pass is the
    synthesis low-pass modulated by (-1)^k, so its Nyquist gain is 1.

The filter bank: the low band is the analysis low-pass centred on even
samples, the high band the analysis high-pass centred on odd samples, over
the whole-sample symmetric extension of the signal (numpy's 'reflect' pad,
which is the symmetric-periodic extension with period 2N-2 for any pad width).
"""
from __future__ import annotations

import numpy as np


def _laurent_mul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Product of two centred (odd-length, symmetric-support) Laurent polynomials."""
    return np.convolve(a, b)


_C = np.array([0.25, 0.5, 0.25])      # cos^2(w/2)
_Y = np.array([-0.25, 0.5, -0.25])    # sin^2(w/2)
_ONE = np.array([1.0])


def _poly_in_y(coeffs_low_first) -> np.ndarray:
    """Evaluate sum_k a_k y^k as a centred Laurent polynomial in z."""
    out = np.zeros(1)
    ypow = _ONE
    for a in coeffs_low_first:
        # pad both to the same centred length before adding
        n = max(out.size, ypow.size)
        o = np.pad(out, ((n - out.size) // 2,) * 2)
        y = np.pad(ypow, ((n - ypow.size) // 2,) * 2)
        out = o + a * y
        ypow = _laurent_mul(ypow, _Y)
    return out


def daubechies_real_root() -> float:
    """The real root of 1 + 4y + 10y^2 + 20y^3."""
    r = np.roots([20.0, 10.0, 4.0, 1.0])
    real = r[np.abs(r.imag) < 1e-12].real
    assert real.size == 1
    return float(real[0])


def cdf_filters(wavelet: str):
    """Return (analysis low-pass h, analysis high-pass g), both centred.

    h has odd length 2*rh+1 and is applied centred on even samples; g has odd
    length 2*rg+1 and is applied centred on odd samples.
    """
    if wavelet == "cdf53":
        syn = _C.copy()                               # 3 taps
        ana = _laurent_mul(_C, _poly_in_y([1.0, 2.0]))  # 5 taps
    elif wavelet == "cdf97":
        yr = daubechies_real_root()
        c2 = _laurent_mul(_C, _C)
        syn = _laurent_mul(c2, _poly_in_y([1.0, -1.0 / yr]))   # 7 taps
        # P4(y) / (1 - y/yr) = -yr * P4(y) / (y - yr): synthetic division
        q, rem = np.polydiv([20.0, 10.0, 4.0, 1.0], [1.0, -yr])
        assert abs(rem[-1]) < 1e-12
        quad_low_first = (-yr * q)[::-1]
        ana = _laurent_mul(c2, _poly_in_y(quad_low_first))   # 9 taps
    else:
        raise ValueError(wavelet)
    k = np.arange(syn.size) - syn.size // 2
    g = ((-1.0) ** k) * syn
    return ana, g


def analysis_1d(x: np.ndarray, wavelet: str, axis: int = -1) -> np.ndarray:
    """One level of the 1-D filter bank along `axis`: [low band | high band]."""
    h, g = cdf_filters(wavelet)
    rh, rg = h.size // 2, g.size // 2
    x = np.moveaxis(np.asarray(x, dtype=np.float64), axis, -1)
    n = x.shape[-1]
    if n < 2 or n % 2:
        raise ValueError("length must be even and >= 2")
    pad = max(rh, rg) + 1
    widths = [(0, 0)] * (x.ndim - 1) + [(pad, pad)]
    xe = np.pad(x, widths, mode="reflect")
    half = n // 2
    low = np.zeros(x.shape[:-1] + (half,))
    high = np.zeros(x.shape[:-1] + (half,))
    for i in range(half):
        c0 = 2 * i + pad
        low[..., i] = xe[..., c0 - rh:c0 + rh + 1] @ h
        c1 = 2 * i + 1 + pad
        high[..., i] = xe[..., c1 - rg:c1 + rg + 1] @ g
    out = np.concatenate([low, high], axis=-1)
    return np.moveaxis(out, -1, axis)


def analysis_2d(x: np.ndarray, wavelet: str, levels: int = 1) -> np.ndarray:
    """L-level 2-D filter bank (rows, then columns), Mallat layout."""
    out = np.array(x, dtype=np.float64, copy=True)
    H, W = out.shape
    for j in range(levels):
        h, w = H >> j, W >> j
        blk = analysis_1d(out[:h, :w], wavelet, axis=1)
        blk = analysis_1d(blk, wavelet, axis=0)
        out[:h, :w] = blk
    return out
