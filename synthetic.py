"""Seeded synthetic inputs for the 2-D DWT workloads.

This module is the only code shared by the GPU library's tests, the benchmark
and the FP64 oracle. It generates inputs and nothing else: no wavelet
arithmetic lives here.

The paper names no image set, so the workloads are synthetic stand-ins with
the sizes and value ranges of 8-bit photographic images:

  * ``uniform_image``   i.i.d. integers 0..255 stored as floats (the hardest
                        case for accuracy: no smoothness, full-range detail);
                        ``device_uniform_image`` draws the same distribution
                        on the GPU;
  * ``sinusoid_image``  a sum of 8 random plane waves (periods 8-512 px) around
                        mid-grey plus Gaussian noise (sigma 4), clipped to
                        0..255: smooth content with texture at many scales;
  * ``batch_sizes``     width and height drawn log-uniformly in [lo, hi],
                        rounded to a multiple of `multiple`;
  * ``request_stream``  a Poisson arrival process of mixed transform requests.

All generators take a seed; the default seed of workload k is SEED_BASE + k.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_BASE = 170508266


def rng_for(config: int, salt: int = 0) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + config + 1000 * salt)


def uniform_image(height: int, width: int, seed: int = SEED_BASE + 1,
                  dtype=np.float32) -> np.ndarray:
    """I.i.d. uniform integers 0..255, as `dtype`."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 256, size=(height, width)).astype(dtype)


def device_uniform_image(height: int, width: int, seed: int, dtype=None, device="cuda"):
    """I.i.d. uniform integers 0..255 drawn directly on a PyTorch device by a
    seeded device generator (for workloads too large to draw on the host; the
    values differ from ``uniform_image`` of the same seed)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    x = torch.randint(0, 256, (height, width), generator=g, device=device, dtype=torch.int32)
    return x.to(dtype or torch.float32)


def sinusoid_image(height: int, width: int, seed: int = SEED_BASE + 2,
                   n_waves: int = 8, amplitude: float = 12.0,
                   noise_sigma: float = 4.0, dtype=np.float32) -> np.ndarray:
    """Sum of random 2-D sinusoids plus Gaussian noise, clipped to 0..255.

    Periods are log-uniform in [8, 512] px, orientations uniform in [0, pi),
    phases uniform in [0, 2 pi). Built row block by row block in float64 so a
    16384^2 image needs no more than a few row blocks of scratch.
    """
    rng = np.random.default_rng(seed)
    periods = np.exp(rng.uniform(math.log(8.0), math.log(512.0), n_waves))
    theta = rng.uniform(0.0, math.pi, n_waves)
    phase = rng.uniform(0.0, 2.0 * math.pi, n_waves)
    out = np.empty((height, width), dtype=dtype)
    xs = np.arange(width, dtype=np.float64)
    block = max(1, min(height, (1 << 22) // max(width, 1)))
    noise_rng = np.random.default_rng(seed + 7)
    for y0 in range(0, height, block):
        ys = np.arange(y0, min(height, y0 + block), dtype=np.float64)[:, None]
        acc = np.full((ys.shape[0], width), 128.0)
        for k in range(n_waves):
            arg = (xs[None, :] * math.cos(theta[k]) + ys * math.sin(theta[k]))
            acc += amplitude * np.sin(2.0 * math.pi * arg / periods[k] + phase[k])
        acc += noise_rng.normal(0.0, noise_sigma, size=acc.shape)
        out[y0:y0 + ys.shape[0]] = np.clip(acc, 0.0, 255.0)
    return out


def batch_sizes(n: int, lo: int = 64, hi: int = 4096, multiple: int = 32,
                seed: int = SEED_BASE + 4):
    """`n` (width, height) pairs, each side exp(U(ln lo, ln hi)) rounded to a
    multiple of `multiple` (at least `multiple`)."""
    rng = np.random.default_rng(seed)
    sides = np.exp(rng.uniform(math.log(lo), math.log(hi), size=(n, 2)))
    sides = np.maximum(multiple, np.round(sides / multiple) * multiple)
    return [(int(w), int(h)) for w, h in sides]


@dataclass
class Request:
    rid: int
    arrival_s: float
    side: int          # square image, side x side pixels
    levels: int
    inverse: bool      # False: forward transform, True: inverse transform
    seed: int


def request_stream(n: int, rate_per_s: float, lo: int = 256, hi: int = 8192,
                   multiple: int = 64, max_levels: int = 6,
                   seed: int = SEED_BASE + 5):
    """Poisson arrivals at `rate_per_s`; side log-uniform in [lo, hi] rounded
    to `multiple`; levels uniform in 1..max_levels; forward or inverse 50/50."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n)
    t = np.cumsum(gaps)
    sides = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n))
    sides = np.maximum(multiple, np.round(sides / multiple) * multiple)
    levels = rng.integers(1, max_levels + 1, size=n)
    inv = rng.random(n) < 0.5
    seeds = rng.integers(0, 2**31 - 1, size=n)
    return [Request(i, float(t[i]), int(sides[i]), int(levels[i]), bool(inv[i]),
                    int(seeds[i])) for i in range(n)]
