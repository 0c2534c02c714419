"""Continuous batching on the GPU: every request's result is the same alone
and in the mix (bit for bit, since each level runs the same per-quad
arithmetic with the same tile configuration), and within the FP16 bound of
the FP64 oracle. Also the level-batch entry points directly."""
import ctypes

import numpy as np
import pytest

import oracle
import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1705_08266_amd as dwt  # noqa: E402
from paper_1705_08266_amd import _lib  # noqa: E402
from paper_1705_08266_amd import serving as sv  # noqa: E402


def _workload(n, seed, lo=64, hi=1024, dtype=torch.float16, rate=5000.0):
    trace = synthetic.request_stream(n, rate, lo=lo, hi=hi, seed=seed)
    reqs, inputs, images = [], {}, {}
    for r in trace:
        img = synthetic.uniform_image(r.side, r.side, seed=r.seed)
        x = torch.from_numpy(img).to("cuda").to(dtype)
        images[r.rid] = x
        # an inverse request's input is the pyramid of a synthetic image
        inputs[r.rid] = dwt.forward(x, "cdf97", r.levels) if r.inverse else x
        reqs.append(sv.Request(r.rid, r.arrival_s, r.side, r.side, r.levels, r.inverse))
    torch.cuda.synchronize()
    return reqs, inputs, images


def _alone(req, x):
    f = dwt.inverse if req.inverse else dwt.forward
    return f(x, "cdf97", req.levels)


def test_results_identical_alone_and_in_the_mix():
    reqs, inputs, images = _workload(40, seed=21)
    total = sum(sv.request_bytes(r) for r in reqs)
    srv = sv.Server(budget_bytes=total // 3, max_active=16)   # admission in waves
    res = srv.run(reqs, inputs, keep_outputs=True, realtime=False)
    torch.cuda.synchronize()
    assert sorted(r.rid for r in res) == sorted(r.rid for r in reqs)
    assert srv.sched.peak_used <= total // 3
    assert srv.iterations < sum(r.levels for r in reqs)       # requests overlapped
    by_id = {r.rid: r for r in reqs}
    for out in res:
        req = by_id[out.rid]
        alone = _alone(req, inputs[req.rid])
        assert torch.equal(alone, out.output), req
        # the same request through a server of its own
        solo = sv.Server().run([req], inputs, keep_outputs=True, realtime=False)[0]
        assert torch.equal(solo.output, out.output), req


@pytest.mark.parametrize("dtype,tdt", [("f32", torch.float32), ("bf16", torch.bfloat16)])
def test_other_storage_types_identical_alone_and_in_the_mix(dtype, tdt):
    reqs, inputs, images = _workload(16, seed=31, hi=768, dtype=tdt)
    srv = sv.Server(dtype=dtype, max_active=6)
    res = srv.run(reqs, inputs, keep_outputs=True, realtime=False)
    torch.cuda.synchronize()
    by_id = {r.rid: r for r in reqs}
    for out in res:
        req = by_id[out.rid]
        assert out.output.dtype == tdt
        assert torch.equal(_alone(req, inputs[req.rid]), out.output), req


def test_server_rejects_inputs_of_another_storage_type():
    reqs, inputs, images = _workload(2, seed=3, hi=256)
    with pytest.raises(ValueError):
        sv.Server(dtype="f32").run(reqs, inputs)


def test_mix_within_fp16_bound_of_the_oracle():
    reqs, inputs, images = _workload(12, seed=5, hi=512)
    res = sv.Server().run(reqs, inputs, keep_outputs=True, realtime=False)
    torch.cuda.synchronize()
    by_id = {r.rid: r for r in reqs}
    for out in res:
        req = by_id[out.rid]
        x64 = inputs[req.rid].float().cpu().numpy().astype(np.float64)
        got = out.output.float().cpu().numpy()
        if req.inverse:
            ref = oracle.inverse(x64, "cdf97", req.levels)
            scale = float(np.abs(images[req.rid].float().cpu().numpy()).max())
        else:
            ref = oracle.forward(x64, "cdf97", req.levels)
            scale = float(np.abs(x64).max())
        assert np.abs(got - ref).max() <= 1e-3 * scale, req


def test_realtime_poisson_run_matches_alone():
    reqs, inputs, images = _workload(24, seed=9, rate=20000.0)
    srv = sv.Server()
    res = srv.run(reqs, inputs, keep_outputs=True, realtime=True)
    torch.cuda.synchronize()
    by_id = {r.rid: r for r in reqs}
    for out in res:
        req = by_id[out.rid]
        assert out.done_s >= out.arrival_s - 1e-3
        assert torch.equal(_alone(req, inputs[req.rid]), out.output)
    assert srv.sched.used == 0


def _bands(pyr, w, h):
    return pyr[:h // 2, w // 2:w], pyr[h // 2:h, :w // 2], pyr[h // 2:h, w // 2:w]


@pytest.mark.parametrize("band_dtype", [torch.float32, torch.float16, torch.bfloat16])
def test_level_batch_equals_single_levels(band_dtype):
    """Mixed sizes (several size classes, more than 36 jobs in one class) and
    mixed FP32/storage-type operands in one call."""
    rng = np.random.default_rng(4)
    lib = dwt.load()
    jobs, expect, got, keep = [], [], [], []
    for i in range(90):
        # 50 jobs of one size class and one type pair, then a mix
        side = 64 if i < 50 else int(rng.choice([64, 96, 160, 640, 2112]))
        h, w = side, side + 32
        full_t = torch.float32 if i >= 50 and i % 3 == 0 else band_dtype
        ll_t = torch.float32 if i >= 50 and i % 2 == 0 else band_dtype
        x = torch.from_numpy(synthetic.uniform_image(h, w, seed=i)).to("cuda").to(full_t)
        pyr = torch.zeros(h, w, device="cuda", dtype=band_dtype)
        ll = torch.zeros(h // 2, w // 2, device="cuda", dtype=ll_t)
        ref_pyr = torch.zeros_like(pyr)
        ref_ll = torch.zeros_like(ll)
        dwt.forward_level(x, ref_ll, *_bands(ref_pyr, w, h))
        jobs.append(sv._job(x, ll, *_bands(pyr, w, h), w, h, dwt._dtype_code))
        keep.append(x)                       # a job holds raw pointers only
        expect.append((ref_pyr, ref_ll))
        got.append((pyr, ll))
    arr = (_lib.LevelJob * len(jobs))(*jobs)
    st = lib.dwt2_forward_level_batch(arr, len(jobs), _lib.CDF97, _lib.NONSEPARABLE, None,
                                      dwt._stream_ptr())
    _lib.check(st)
    torch.cuda.synchronize()
    for (ep, el), (gp, gl) in zip(expect, got):
        h, w = ep.shape
        for a, b in zip(_bands(ep, w, h), _bands(gp, w, h)):
            assert torch.equal(a, b)
        assert torch.equal(el, gl)
    # inverse of every job in one call equals the single-level inverse
    inv_jobs, inv_expect, inv_got = [], [], []
    for (gp, gl) in got:
        h, w = gp.shape
        out = torch.zeros(h, w, device="cuda", dtype=torch.float32)
        ref = torch.zeros_like(out)
        dwt.inverse_level(gl, *_bands(gp, w, h), ref)
        inv_jobs.append(sv._job(out, gl, *_bands(gp, w, h), w, h, dwt._dtype_code))
        inv_expect.append(ref)
        inv_got.append(out)
    arr = (_lib.LevelJob * len(inv_jobs))(*inv_jobs)
    _lib.check(lib.dwt2_inverse_level_batch(arr, len(inv_jobs), _lib.CDF97, _lib.NONSEPARABLE,
                                            None, dwt._stream_ptr()))
    torch.cuda.synchronize()
    for a, b in zip(inv_expect, inv_got):
        assert torch.equal(a, b)


def test_level_batch_rejects_bad_job_before_launch():
    lib = dwt.load()
    x = torch.zeros(64, 64, device="cuda")
    pyr = torch.full((64, 64), 7.0, device="cuda")
    ll = torch.zeros(32, 32, device="cuda")
    good = sv._job(x, ll, *_bands(pyr, 64, 64), 64, 64, dwt._dtype_code)
    bad = sv._job(x, ll, *_bands(pyr, 64, 64), 64, 64, dwt._dtype_code)
    bad.full_pitch = 32                               # row pitch below the width
    arr = (_lib.LevelJob * 2)(good, bad)
    st = lib.dwt2_forward_level_batch(arr, 2, _lib.CDF97, _lib.NONSEPARABLE, None,
                                      dwt._stream_ptr())
    assert st == _lib.ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert bool((pyr == 7.0).all())                   # nothing was launched
    tiles = (ctypes.c_int32 * 4)(4, 4, 4, 4)          # a stream configuration: not batchable
    st = lib.dwt2_forward_level_batch(arr, 1, _lib.CDF97, _lib.NONSEPARABLE, tiles,
                                      dwt._stream_ptr())
    assert st == _lib.ERR_UNSUPPORTED
    assert lib.dwt2_forward_level_batch(arr, 0, _lib.CDF97, _lib.NONSEPARABLE, None,
                                        dwt._stream_ptr()) == _lib.OK
