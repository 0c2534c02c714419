"""FP64 oracle for the 2-D CDF 9/7 and CDF 5/3 discrete wavelet transform.

TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package. It shares no code with the GPU
library (``paper_1705_08266_amd``) and imports nothing from it; the only module
the two sides share is the seeded input generator ``synthetic``, which holds no
transform arithmetic.

Contents
  * ``dwt2_ref.c``      plain separable lifting, FP64 (built as ``liboracle_dwt2.so``)
  * ``filterbank.py``   closed-form CDF filters and a direct-convolution filter bank
  * ``nonsep_model.py`` the paper's non-separable lifting in its matrix notation

The C library is wrapped here with ctypes: :func:`forward`, :func:`inverse`,
:func:`forward_1d`, :func:`inverse_1d`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle_dwt2.so")
SRC_PATH = os.path.join(_HERE, "dwt2_ref.c")

CDF97 = 0
CDF53 = 1
WAVELETS = {"cdf97": CDF97, "cdf53": CDF53}

_lib = None


def build(verbose: bool = False) -> str:
    """Compile the C oracle with the host compiler (-O2, no fast-math, OpenMP)."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c99",
           "-Wall", "-Wextra", "-o", LIB_PATH + ".tmp", SRC_PATH]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH) or (
            os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH)):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    for name in ("oracle_dwt2_forward", "oracle_dwt2_inverse"):
        f = getattr(lib, name)
        f.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                      ctypes.c_int, ctypes.c_int]
        f.restype = ctypes.c_int
    for name in ("oracle_dwt1_forward", "oracle_dwt1_inverse"):
        f = getattr(lib, name)
        f.argtypes = [dp, ctypes.c_int, ctypes.c_int]
        f.restype = ctypes.c_int
    lib.oracle_max_threads.argtypes = []
    lib.oracle_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _wid(wavelet) -> int:
    if isinstance(wavelet, str):
        return WAVELETS[wavelet]
    return int(wavelet)


def _as_f64(x: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.float64)


def max_threads() -> int:
    return _load().oracle_max_threads()


def forward(x: np.ndarray, wavelet="cdf97", levels: int = 1,
            nthreads: int = 1) -> np.ndarray:
    """L-level forward DWT of a 2-D image (H rows x W columns), Mallat layout."""
    lib = _load()
    src = _as_f64(x)
    if src.ndim != 2:
        raise ValueError("expected a 2-D image")
    H, W = src.shape
    out = np.empty_like(src)
    dp = ctypes.POINTER(ctypes.c_double)
    st = lib.oracle_dwt2_forward(src.ctypes.data_as(dp), out.ctypes.data_as(dp),
                                 W, H, _wid(wavelet), int(levels), int(nthreads))
    if st != 0:
        raise ValueError(f"oracle forward rejected W={W} H={H} levels={levels}")
    return out


def inverse(c: np.ndarray, wavelet="cdf97", levels: int = 1,
            nthreads: int = 1) -> np.ndarray:
    """Inverse of :func:`forward`."""
    lib = _load()
    src = _as_f64(c)
    if src.ndim != 2:
        raise ValueError("expected a 2-D coefficient array")
    H, W = src.shape
    out = np.empty_like(src)
    dp = ctypes.POINTER(ctypes.c_double)
    st = lib.oracle_dwt2_inverse(src.ctypes.data_as(dp), out.ctypes.data_as(dp),
                                 W, H, _wid(wavelet), int(levels), int(nthreads))
    if st != 0:
        raise ValueError(f"oracle inverse rejected W={W} H={H} levels={levels}")
    return out


def forward_1d(x: np.ndarray, wavelet="cdf97") -> np.ndarray:
    """One-level 1-D forward transform: returns [low band | high band]."""
    lib = _load()
    y = _as_f64(x).copy()
    dp = ctypes.POINTER(ctypes.c_double)
    if lib.oracle_dwt1_forward(y.ctypes.data_as(dp), y.size, _wid(wavelet)) != 0:
        raise ValueError("oracle 1-D forward rejected its input")
    return y


def inverse_1d(x: np.ndarray, wavelet="cdf97") -> np.ndarray:
    lib = _load()
    y = _as_f64(x).copy()
    dp = ctypes.POINTER(ctypes.c_double)
    if lib.oracle_dwt1_inverse(y.ctypes.data_as(dp), y.size, _wid(wavelet)) != 0:
        raise ValueError("oracle 1-D inverse rejected its input")
    return y


def subbands(coef: np.ndarray, level: int, levels: int):
    """Views (LL or None, HL, LH, HH) of level `level` (1-based) in a Mallat array."""
    H, W = coef.shape
    h, w = H >> level, W >> level
    hl = coef[:h, w:2 * w]
    lh = coef[h:2 * h, :w]
    hh = coef[h:2 * h, w:2 * w]
    ll = coef[:h, :w] if level == levels else None
    return ll, hl, lh, hh
