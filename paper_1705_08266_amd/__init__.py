"""2-D CDF 9/7 and CDF 5/3 DWT on MI355X by non-separable lifting.

Thin binding over the C ABI of ``libdwt2.so`` (include/dwt2.h). Every step of
the transform runs in the library's HIP kernels; this module only checks
tensors, marshals pointers and picks the current HIP stream. PyTorch serves
for device memory and streams.

    import torch, paper_1705_08266_amd as dwt
    x = torch.rand(4096, 4096, device="cuda") * 255
    c = dwt.forward(x, "cdf97", levels=5)            # Mallat layout, same shape
    y = dwt.inverse(c, "cdf97", levels=5)
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import DWT2Error, load  # noqa: F401

WAVELETS = {"cdf97": _lib.CDF97, "cdf53": _lib.CDF53}
SCHEMES = {"nonseparable": _lib.NONSEPARABLE, "separable": _lib.SEPARABLE,
           # every neighbour exchange through LDS: the barrier-count ablation
           "nonseparable_lds": _lib.NONSEPARABLE_LDS, "separable_lds": _lib.SEPARABLE_LDS}


def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    codes = {torch.float32: _lib.F32, torch.float16: _lib.F16, torch.bfloat16: _lib.BF16}
    if t.dtype not in codes:
        raise TypeError(f"unsupported dtype {t.dtype}; use float32, float16 or bfloat16")
    return codes[t.dtype]


def _check_2d(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be 2-D with unit stride along rows")


def _desc(t) -> _lib.Desc:
    return _lib.Desc(t.shape[1], t.shape[0], t.stride(0), _dtype_code(t))


def _wavelet(w) -> int:
    return WAVELETS[w] if isinstance(w, str) else int(w)


def _scheme(s) -> int:
    return SCHEMES[s] if isinstance(s, str) else int(s)


def _stream_ptr(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _tiles_arg(tiles, levels):
    if tiles is None:
        return None
    if len(tiles) != levels:
        raise ValueError("need one tile id per level")
    return (ctypes.c_int32 * levels)(*[int(t) for t in tiles])


def _events_arg(events, levels):
    if events is None:
        return None
    if len(events) != 2 * levels:
        raise ValueError("need two events per level")
    for e in events:
        if not e.cuda_event:     # PyTorch creates the HIP event on its first record
            e.record()
    return (ctypes.c_void_p * (2 * levels))(*[e.cuda_event for e in events])


def workspace_bytes(width: int, height: int, levels: int, dtype=_lib.F32) -> int:
    """Workspace bytes of an L-level transform (the same for every storage
    type: intermediate low-low bands are FP32)."""
    return int(load().dwt2_workspace_bytes(width, height, levels, int(dtype)))


def make_workspace(width: int, height: int, levels: int, device=None):
    torch = _torch()
    n = workspace_bytes(width, height, levels)
    return torch.empty(max(1, n // 4), dtype=torch.float32, device=device or "cuda")


def forward(x, wavelet="cdf97", levels: int = 1, scheme="nonseparable", out=None,
            workspace=None, tiles=None, events=None, stream=None):
    """L-level forward DWT of a 2-D GPU image; returns the Mallat-layout
    coefficients (same shape and dtype)."""
    torch = _torch()
    _check_2d(x, "x")
    if out is None:
        out = torch.empty_like(x)
    _check_2d(out, "out")
    H, W = x.shape
    if workspace is None and workspace_bytes(W, H, levels) > 0:
        workspace = make_workspace(W, H, levels, x.device)
    ws_ptr = workspace.data_ptr() if workspace is not None else None
    ws_n = workspace.numel() * workspace.element_size() if workspace is not None else 0
    dx, do = _desc(x), _desc(out)
    args = (x.data_ptr(), ctypes.byref(dx), out.data_ptr(), ctypes.byref(do),
            _wavelet(wavelet), levels, _lib.EXT_WHOLE_SAMPLE_SYMMETRIC, _scheme(scheme),
            ws_ptr, ws_n)
    if tiles is None and events is None:
        st = load().dwt2_forward(*args, _stream_ptr(stream))
    else:
        st = load().dwt2_forward_ex(*args, _tiles_arg(tiles, levels),
                                    _events_arg(events, levels), _stream_ptr(stream))
    _lib.check(st, "dwt2_forward")
    return out


def forward_no_alloc(x, out, wavelet="cdf97", levels: int = 1, scheme="nonseparable",
                     stream=None):
    """:func:`forward` into a caller-provided `out`, with the library's own
    device workspace: the call allocates nothing (for graph capture and
    allocation-free loops). Calls on one GPU share that workspace and must not
    overlap in time."""
    _check_2d(x, "x")
    _check_2d(out, "out")
    dx, do = _desc(x), _desc(out)
    st = load().dwt2_forward_no_alloc(x.data_ptr(), ctypes.byref(dx), out.data_ptr(),
                                      ctypes.byref(do), _wavelet(wavelet), levels,
                                      _lib.EXT_WHOLE_SAMPLE_SYMMETRIC, _scheme(scheme),
                                      _stream_ptr(stream))
    _lib.check(st, "dwt2_forward_no_alloc")
    return out


def inverse(c, wavelet="cdf97", levels: int = 1, scheme="nonseparable", out=None,
            workspace=None, tiles=None, events=None, stream=None):
    """Inverse of :func:`forward`."""
    torch = _torch()
    _check_2d(c, "c")
    if out is None:
        out = torch.empty_like(c)
    _check_2d(out, "out")
    H, W = c.shape
    if workspace is None and workspace_bytes(W, H, levels) > 0:
        workspace = make_workspace(W, H, levels, c.device)
    ws_ptr = workspace.data_ptr() if workspace is not None else None
    ws_n = workspace.numel() * workspace.element_size() if workspace is not None else 0
    dc, do = _desc(c), _desc(out)
    args = (c.data_ptr(), ctypes.byref(dc), out.data_ptr(), ctypes.byref(do),
            _wavelet(wavelet), levels, _lib.EXT_WHOLE_SAMPLE_SYMMETRIC, _scheme(scheme),
            ws_ptr, ws_n)
    if tiles is None and events is None:
        st = load().dwt2_inverse(*args, _stream_ptr(stream))
    else:
        st = load().dwt2_inverse_ex(*args, _tiles_arg(tiles, levels),
                                    _events_arg(events, levels), _stream_ptr(stream))
    _lib.check(st, "dwt2_inverse")
    return out


def forward_level(x, ll, hl, lh, hh, wavelet="cdf97", scheme="nonseparable", tile=-1,
                  stream=None):
    """One level: x (H x W) -> four (H/2 x W/2) bands. hl, lh and hh must share
    one row pitch (e.g. views into a Mallat array)."""
    for t, n in ((x, "x"), (ll, "ll"), (hl, "hl"), (lh, "lh"), (hh, "hh")):
        _check_2d(t, n)
    if not (hl.stride(0) == lh.stride(0) == hh.stride(0)):
        raise ValueError("hl, lh and hh must share a row pitch")
    H, W = x.shape
    st = load().dwt2_forward_level(
        x.data_ptr(), x.stride(0), _dtype_code(x), W, H,
        ll.data_ptr(), ll.stride(0), _dtype_code(ll),
        hl.data_ptr(), lh.data_ptr(), hh.data_ptr(), hl.stride(0), _dtype_code(hl),
        _wavelet(wavelet), _scheme(scheme), int(tile), _stream_ptr(stream))
    _lib.check(st, "dwt2_forward_level")


def inverse_level(ll, hl, lh, hh, out, wavelet="cdf97", scheme="nonseparable", tile=-1,
                  stream=None):
    for t, n in ((out, "out"), (ll, "ll"), (hl, "hl"), (lh, "lh"), (hh, "hh")):
        _check_2d(t, n)
    if not (hl.stride(0) == lh.stride(0) == hh.stride(0)):
        raise ValueError("hl, lh and hh must share a row pitch")
    H, W = out.shape
    st = load().dwt2_inverse_level(
        ll.data_ptr(), ll.stride(0), _dtype_code(ll),
        hl.data_ptr(), lh.data_ptr(), hh.data_ptr(), hl.stride(0), _dtype_code(hl),
        out.data_ptr(), out.stride(0), _dtype_code(out), W, H,
        _wavelet(wavelet), _scheme(scheme), int(tile), _stream_ptr(stream))
    _lib.check(st, "dwt2_inverse_level")


def tile_configs(wavelet="cdf97"):
    """[(id, quads_per_lane, rows, waves, out_x, out_y)] compiled in."""
    lib = load()
    out = []
    for t in range(lib.dwt2_tile_config_count()):
        v = [ctypes.c_int32() for _ in range(5)]
        _lib.check(lib.dwt2_tile_config_info(t, _wavelet(wavelet), *[ctypes.byref(a) for a in v]))
        out.append((t, *[a.value for a in v]))
    return out


def fused_levels(width: int, height: int, levels: int) -> int:
    """Trailing levels the library runs as one fused launch by default."""
    n = int(load().dwt2_fused_levels(width, height, levels))
    _lib.check(min(n, 0), "dwt2_fused_levels")
    return n


def head_levels(width: int, height: int, levels: int) -> int:
    """Leading levels (0 or 2) the library runs as one fused launch by default."""
    n = int(load().dwt2_head_levels(width, height, levels))
    _lib.check(min(n, 0), "dwt2_head_levels")
    return n


def default_tile(width, height, wavelet="cdf97", scheme="nonseparable", dtype=_lib.F32):
    return int(load().dwt2_default_tile(width, height, _wavelet(wavelet), _scheme(scheme), dtype))
