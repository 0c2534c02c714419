"""Batches of uneven images, planned once and run as one launch per level
(per tile configuration in use), capturable as one HIP graph.

    plan = BatchPlan.forward(images, levels=3)     # list of 2-D GPU tensors
    plan.capture()                                 # record the launches once
    plan.replay()                                  # one graph launch per call
    coefs = plan.outputs

The library plans the launch table (dwt2_batch_plan) in host memory; this
module copies it to a device tensor and hands both copies to dwt2_batch_run,
whose kernels read the per-tile image map and level parameters from device
memory. Every transform step runs in the library's kernels; this module
allocates outputs, workspaces and the plan's device copy with PyTorch.
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


def make_plan(srcs, dsts, workspaces, inverse=False, wavelet="cdf97", levels=1,
              class_tiles=None, fuse_head=False):
    """The host plan of a batched transform srcs[i] -> dsts[i] (a ctypes byte
    buffer). fuse_head: levels 1 and 2 of every image in one head launch."""
    if not (len(srcs) == len(dsts) == len(workspaces)) or not srcs:
        raise ValueError("need one dst and one workspace per src, and at least one image")
    dt = _dtype_code(srcs[0])
    for s, d in zip(srcs, dsts):
        if not (s.is_cuda and d.is_cuda) or s.dim() != 2 or s.stride(1) != 1 or d.stride(1) != 1:
            raise ValueError("batch images must be 2-D GPU tensors with unit row stride")
        if _dtype_code(s) != dt or _dtype_code(d) != dt or s.shape != d.shape:
            raise ValueError("all batch images share one dtype; dst matches src")
    arr = _image_array(srcs, dsts, workspaces)
    lib = load()
    args = (arr, len(srcs), dt, _wavelet(wavelet), int(levels), int(bool(inverse)),
            _lib.EXT_WHOLE_SAMPLE_SYMMETRIC, _class_tiles(class_tiles),
            _lib.PLAN_HEAD if fuse_head else 0)
    n = ctypes.c_size_t()
    _lib.check(lib.dwt2_batch_plan_bytes(*args, ctypes.byref(n)), "dwt2_batch_plan_bytes")
    buf = (ctypes.c_ubyte * n.value)()
    _lib.check(lib.dwt2_batch_plan(*args, buf, n.value), "dwt2_batch_plan")
    return buf


class BatchPlan:
    """A fixed batch of images with outputs, workspaces and the plan's device
    copy allocated once; run() enqueues it, capture()/replay() use a graph."""

    def __init__(self, srcs, inverse, wavelet, levels, scheme, class_tiles, persistent=False,
                 fuse_head=False):
        import torch
        self.srcs = list(srcs)
        self.inverse = inverse
        self.wavelet, self.levels, self.scheme = wavelet, levels, scheme
        self.class_tiles = class_tiles
        self.persistent = persistent
        self.fuse_head = fuse_head
        self.outputs = [torch.empty_like(s) for s in self.srcs]
        self.workspaces = [
            torch.empty(max(1, workspace_bytes(s.shape[1], s.shape[0], levels) // 4),
                        dtype=torch.float32, device=s.device) for s in self.srcs]
        self.host_plan = make_plan(self.srcs, self.outputs, self.workspaces, inverse, wavelet,
                                   levels, class_tiles, fuse_head)
        host = torch.frombuffer(bytearray(self.host_plan), dtype=torch.uint8)
        self.device_plan = host.to(self.srcs[0].device)
        torch.cuda.synchronize()
        self.graph = None

    @classmethod
    def forward(cls, images, levels=1, wavelet="cdf97", scheme="nonseparable", class_tiles=None,
                persistent=False, fuse_head=False):
        return cls(images, False, wavelet, levels, scheme, class_tiles, persistent, fuse_head)

    @classmethod
    def inverse_of(cls, coefs, levels=1, wavelet="cdf97", scheme="nonseparable",
                   class_tiles=None, persistent=False, fuse_head=False):
        return cls(coefs, True, wavelet, levels, scheme, class_tiles, persistent, fuse_head)

    def launches(self):
        """(total launches, launches per level j = 1..L)."""
        total = ctypes.c_int32()
        per = (ctypes.c_int32 * self.levels)()
        _lib.check(load().dwt2_batch_launches(self.host_plan, len(self.host_plan),
                                              ctypes.byref(total), per), "dwt2_batch_launches")
        return total.value, list(per)

    def run(self, stream=None):
        st = load().dwt2_batch_run(self.host_plan, len(self.host_plan),
                                   self.device_plan.data_ptr(), _scheme(self.scheme),
                                   _lib.BATCH_PERSISTENT if self.persistent else 0,
                                   _stream_ptr(stream))
        _lib.check(st, "dwt2_batch_run")

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
