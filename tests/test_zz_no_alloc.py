"""dwt2_forward_no_alloc against dwt2_forward, both through the C ABI.

The no-alloc call takes its workspace from the library's own device array;
results must be identical to dwt2_forward with a caller workspace (the same
kernels on the same values). Two calls in a row, the second on a smaller
input, show that nothing left in the shared array from one call reaches the
next."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1705_08266_amd import _lib
import synthetic

pytestmark = pytest.mark.gpu

_CODES = {torch.float32: _lib.F32, torch.float16: _lib.F16, torch.bfloat16: _lib.BF16}


def _desc(t):
    return _lib.Desc(t.shape[1], t.shape[0], t.stride(0), _CODES[t.dtype])


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _forward(x, wavelet, levels, scheme):
    lib = _lib.load()
    out = torch.empty_like(x)
    need = lib.dwt2_workspace_bytes(x.shape[1], x.shape[0], levels, _CODES[x.dtype])
    ws = torch.empty(max(1, need // 4), dtype=torch.float32, device=x.device)
    dx, do = _desc(x), _desc(out)
    st = lib.dwt2_forward(x.data_ptr(), ctypes.byref(dx), out.data_ptr(), ctypes.byref(do),
                          wavelet, levels, 0, scheme, ws.data_ptr(), need, _stream())
    assert st == _lib.OK, st
    return out


def _no_alloc(x, out, wavelet, levels, scheme):
    lib = _lib.load()
    dx, do = _desc(x), _desc(out)
    return lib.dwt2_forward_no_alloc(x.data_ptr(), ctypes.byref(dx), out.data_ptr(),
                                     ctypes.byref(do), wavelet, levels, 0, scheme, _stream())


CASES = [   # (first call, second call): the second input is smaller
    (((4096, 4096), 5, torch.float32), ((512, 384), 3, torch.float32)),
    (((1088, 1920), 4, torch.float16), ((256, 192), 2, torch.float16)),
    (((2048, 1024), 6, torch.float32), ((96, 64), 5, torch.float32)),
]


@pytest.mark.parametrize("wavelet", [_lib.CDF97, _lib.CDF53])
@pytest.mark.parametrize("scheme", [_lib.NONSEPARABLE, _lib.SEPARABLE])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_no_alloc_matches_forward_on_two_calls(case, scheme, wavelet):
    outs = []
    for k, ((h, w), levels, dt) in enumerate(CASES[case]):
        print(f"no_alloc case {case} call {k}: {w}x{h} L={levels} {dt} scheme {scheme} "
              f"wavelet {wavelet}", flush=True)
        x = torch.from_numpy(synthetic.uniform_image(h, w, seed=synthetic.SEED_BASE + 40 + k)
                             ).to("cuda", dt)
        out = torch.full_like(x, float("nan"))
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        st = _no_alloc(x, out, wavelet, levels, scheme)
        assert st == _lib.OK, st
        assert torch.cuda.memory_allocated() == before
        want = _forward(x, wavelet, levels, scheme)
        torch.cuda.synchronize()
        assert torch.equal(out, want), (case, k)
        outs.append(out)
    assert len(outs) == 2


def test_no_alloc_refuses_more_than_its_workspace():
    lib = _lib.load()
    x = torch.zeros(16384, 16384, dtype=torch.float16, device="cuda")
    out = torch.zeros_like(x)
    assert lib.dwt2_workspace_bytes(16384, 16384, 5, _lib.F16) > _lib.STATIC_WORKSPACE_BYTES
    assert _no_alloc(x, out, _lib.CDF97, 5, _lib.NONSEPARABLE) == _lib.ERR_WORKSPACE
    # one level needs no workspace at all
    assert _no_alloc(x, out, _lib.CDF97, 1, _lib.NONSEPARABLE) == _lib.OK
    torch.cuda.synchronize()
    assert torch.equal(out, torch.zeros_like(out))
