"""Batches of uneven images: one launch per level and size class, captured
as one HIP graph.

    plan = BatchPlan.forward(images, levels=3)     # list of 2-D GPU tensors
    plan.capture()                                 # record the whole chain once
    plan.replay()                                  # one graph launch per call
    coefs = plan.outputs

Every transform step runs in the library's batched kernels
(dwt2_forward_batch / dwt2_inverse_batch); this module allocates outputs and
workspaces with PyTorch and marshals descriptors.
"""
from __future__ import annotations

import ctypes

from . import _lib
from . import _dtype_code, _scheme, _stream_ptr, _wavelet, load, workspace_bytes


def size_class(width: int, height: int) -> int:
    return int(load().dwt2_size_class(width, height))


def _image_array(srcs, dsts, wss):
    arr = (_lib.Image * len(srcs))()
    for i, (s, d, w) in enumerate(zip(srcs, dsts, wss)):
        arr[i].src = s.data_ptr()
        arr[i].src_pitch = s.stride(0)
        arr[i].dst = d.data_ptr()
        arr[i].dst_pitch = d.stride(0)
        arr[i].workspace = w.data_ptr() if w is not None else None
        arr[i].workspace_bytes = w.numel() * w.element_size() if w is not None else 0
        arr[i].width = s.shape[1]
        arr[i].height = s.shape[0]
    return arr


def _class_tiles(class_tiles):
    if class_tiles is None:
        return None
    if len(class_tiles) != _lib.SIZE_CLASSES:
        raise ValueError(f"need {_lib.SIZE_CLASSES} tile ids, one per size class")
    return (ctypes.c_int32 * _lib.SIZE_CLASSES)(*[int(t) for t in class_tiles])


def run_batch(srcs, dsts, workspaces, inverse=False, wavelet="cdf97", levels=1,
              scheme="nonseparable", class_tiles=None, stream=None):
    """Enqueue one batched transform of srcs[i] -> dsts[i]."""
    if not (len(srcs) == len(dsts) == len(workspaces)):
        raise ValueError("srcs, dsts and workspaces must have the same length")
    if not srcs:
        return
    dt = _dtype_code(srcs[0])
    for s, d in zip(srcs, dsts):
        if not (s.is_cuda and d.is_cuda) or s.dim() != 2 or s.stride(1) != 1 or d.stride(1) != 1:
            raise ValueError("batch images must be 2-D GPU tensors with unit row stride")
        if _dtype_code(s) != dt or _dtype_code(d) != dt or s.shape != d.shape:
            raise ValueError("all batch images share one dtype; dst matches src")
    arr = _image_array(srcs, dsts, workspaces)
    fn = load().dwt2_inverse_batch if inverse else load().dwt2_forward_batch
    st = fn(arr, len(srcs), dt, _wavelet(wavelet), int(levels), _lib.EXT_WHOLE_SAMPLE_SYMMETRIC,
            _scheme(scheme), _class_tiles(class_tiles), _stream_ptr(stream))
    _lib.check(st, "dwt2_inverse_batch" if inverse else "dwt2_forward_batch")


class BatchPlan:
    """A fixed batch of images with its outputs and workspaces allocated once;
    the batched launches can be captured in a HIP graph and replayed."""

    def __init__(self, srcs, inverse, wavelet, levels, scheme, class_tiles):
        import torch
        self.srcs = list(srcs)
        self.inverse = inverse
        self.wavelet, self.levels, self.scheme = wavelet, levels, scheme
        self.class_tiles = class_tiles
        self.outputs = [torch.empty_like(s) for s in self.srcs]
        self.workspaces = [
            torch.empty(max(1, workspace_bytes(s.shape[1], s.shape[0], levels) // 4),
                        dtype=torch.float32, device=s.device) for s in self.srcs]
        self.graph = None

    @classmethod
    def forward(cls, images, levels=1, wavelet="cdf97", scheme="nonseparable", class_tiles=None):
        return cls(images, False, wavelet, levels, scheme, class_tiles)

    @classmethod
    def inverse_of(cls, coefs, levels=1, wavelet="cdf97", scheme="nonseparable", class_tiles=None):
        return cls(coefs, True, wavelet, levels, scheme, class_tiles)

    def run(self, stream=None):
        run_batch(self.srcs, self.outputs, self.workspaces, self.inverse, self.wavelet,
                  self.levels, self.scheme, self.class_tiles, stream)

    def capture(self):
        import torch
        self.run()                      # eager once (and validates arguments)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            self.capture()
        self.graph.replay()

    @property
    def pixels(self) -> int:
        return sum(s.shape[0] * s.shape[1] for s in self.srcs)
