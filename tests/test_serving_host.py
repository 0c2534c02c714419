"""Host logic of the serving loop: admission, level-synchronous iterations and
per-level job descriptors, checked on the CPU with a simulated clock."""
import math

import numpy as np
import pytest

import synthetic
from paper_1705_08266_amd import _lib
from paper_1705_08266_amd import serving as sv

torch = pytest.importorskip("torch")


def _trace(n, seed=3, rate=2000.0, lo=64, hi=2048):
    return [sv.Request(r.rid, r.arrival_s, r.side, r.side, r.levels, r.inverse)
            for r in synthetic.request_stream(n, rate, lo=lo, hi=hi, seed=seed)]


def simulate(requests, budget, max_active=1 << 30, bw=4e12, launch_s=5e-6):
    """Fake executor: one iteration costs a launch overhead plus the bytes of
    the levels it advances at `bw`. Returns per-request admission iteration,
    completion time and the ordered log of (iteration, rid, level)."""
    sched = sv.Scheduler(budget, max_active)
    pending = sorted(requests, key=lambda r: r.arrival_s)
    now, it, k = 0.0, 0, 0
    admitted_at, done_at, log, order = {}, {}, [], []
    while k < len(pending) or not sched.idle:
        while k < len(pending) and pending[k].arrival_s <= now:
            sched.offer(pending[k])
            k += 1
        for a in sched.admit(now):
            assert a.req.arrival_s <= now
            admitted_at[a.req.rid] = it
            order.append(a.req.rid)
        assert sched.used <= budget
        adv = sched.iteration()
        if not adv:
            now = pending[k].arrival_s if k < len(pending) else now
            continue
        cost = launch_s
        for a in adv:
            j = a.next_level + 1
            px = a.req.width * a.req.height / 4 ** (j - 1)
            cost += 6.5 * px / bw
            log.append((it, a.req.rid, a.next_level))
        now += cost
        for a in sched.finish_iteration(adv):
            done_at[a.req.rid] = (it, now)
            sched.release(a)
        it += 1
    return sched, admitted_at, done_at, log, order


def test_every_request_advances_once_per_iteration_until_done():
    reqs = _trace(200)
    sched, adm, done, log, order = simulate(reqs, budget=2 << 30)
    assert not sched.rejected and sched.used == 0
    for r in reqs:
        steps = [(it, lv) for it, rid, lv in log if rid == r.rid]
        # levels 0..L-1 in consecutive iterations starting at admission
        assert [lv for _, lv in steps] == list(range(r.levels))
        assert [it for it, _ in steps] == list(range(adm[r.rid], adm[r.rid] + r.levels))
        assert done[r.rid][0] == adm[r.rid] + r.levels - 1


def test_admission_is_fifo_and_within_budget():
    reqs = _trace(300, seed=8, rate=1e6)           # heavy overload
    budget = 256 << 20
    sched, adm, done, log, order = simulate(reqs, budget=budget)
    arrival_order = [r.rid for r in sorted(reqs, key=lambda r: r.arrival_s)
                     if sv.request_bytes(r) <= budget]
    assert order == arrival_order
    assert sched.peak_used <= budget
    assert sched.peak_used > budget // 2           # the budget is actually used


def test_max_active_is_respected():
    reqs = _trace(100, seed=4, rate=1e6)
    sched = sv.Scheduler(1 << 40, max_active=7)
    for r in reqs:
        sched.offer(r)
    while not sched.idle:
        sched.admit(0.0)
        assert len(sched.active) <= 7
        for a in sched.finish_iteration(sched.iteration()):
            sched.release(a)


def test_oversized_request_is_rejected_and_others_served():
    big = sv.Request(0, 0.0, 8192, 8192, 3, False)
    small = sv.Request(1, 0.0, 256, 256, 2, True)
    sched, adm, done, log, order = simulate([big, small], budget=64 << 20)
    assert [r.rid for r in sched.rejected] == [0]
    assert 1 in done and 0 not in done


def test_small_request_overtakes_a_long_one_in_flight():
    """Continuous batching: a one-level request that arrives while a six-level
    request is running finishes first."""
    long_ = sv.Request(0, 0.0, 4096, 4096, 6, False)
    short = sv.Request(1, 1e-6, 256, 256, 1, False)
    sched, adm, done, log, order = simulate([long_, short], budget=1 << 30)
    assert adm[1] == 1 and done[1][0] == 1
    assert done[0][0] == 5
    assert done[1][1] < done[0][1]


def test_request_bytes_formula():
    r = sv.Request(0, 0.0, 1024, 512, 5, False)
    px = 1024 * 512
    assert sv.request_bytes(r, _lib.F16) == 4 * px + 4 * (px // 4 + px // 16)
    assert sv.request_bytes(r, _lib.F32) == 8 * px + 4 * (px // 4 + px // 16)
    assert sv.workspace_bytes(1024, 512, 1) == 0
    assert sv.workspace_bytes(1024, 512, 2) == px


@pytest.mark.parametrize("inverse", [False, True])
@pytest.mark.parametrize("levels", [1, 2, 3, 5])
def test_level_jobs_chain_and_layout(inverse, levels):
    H, W = 96, 128
    src = torch.zeros(H, W, dtype=torch.float16)
    out = torch.zeros(H, W, dtype=torch.float16)
    ws0 = torch.zeros(max(1, (W // 2) * (H // 2)), dtype=torch.float32)
    ws1 = torch.zeros(max(1, (W // 4) * (H // 4)), dtype=torch.float32)
    jobs = sv.level_jobs(src, out, ws0, ws1, levels, inverse)
    assert len(jobs) == levels
    pyr = src if inverse else out
    e = 2
    bufs = {ws0.data_ptr(): ws0.numel(), ws1.data_ptr(): ws1.numel()}
    lv = list(range(levels, 0, -1)) if inverse else list(range(1, levels + 1))
    for k, (j, job) in enumerate(zip(lv, jobs)):
        h, w = H >> (j - 1), W >> (j - 1)
        assert (job.width, job.height) == (w, h)
        base = pyr.data_ptr()
        assert job.hl == base + e * (w // 2)
        assert job.lh == base + e * (h // 2) * W
        assert job.hh == base + e * ((h // 2) * W + w // 2)
        assert job.band_pitch == W and job.band_dtype == _lib.F16
        for ptr, pitch, dt, n in ((job.full, job.full_pitch, job.full_dtype, h * w),
                                  (job.ll, job.ll_pitch, job.ll_dtype, h * w // 4)):
            if ptr in bufs:                        # an FP32 intermediate fits its buffer
                assert dt == _lib.F32 and n <= bufs[ptr]
                assert pitch == (w if n == h * w else w // 2)
        # the image side of level 1 and the pyramid's LL at level L
        if j == 1:
            assert job.full == (out if inverse else src).data_ptr() and job.full_pitch == W
        if j == levels:
            assert job.ll == base and job.ll_pitch == W and job.ll_dtype == _lib.F16
        else:
            assert job.ll in bufs
    # consecutive levels hand over the LL buffer
    for a, b in zip(jobs, jobs[1:]):
        if inverse:
            assert a.full == b.ll
        else:
            assert a.ll == b.full
        assert a.full != a.ll


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert sv.percentile(v, 50) == 50
    assert sv.percentile(v, 99) == 99
    assert sv.percentile(v, 100) == 100
    assert sv.percentile([3.0], 99) == 3.0
    assert math.isclose(sv.percentile(np.linspace(0, 1, 11).tolist(), 50), 0.5)


def test_percentile_is_exact_at_99_9():
    v = list(range(1, 1001))
    assert sv.percentile(v, 99.9) == 999          # ceil(0.999 * 1000) = 999, not 1000
    assert sv.percentile(v, 99) == 990
    assert sv.percentile(list(range(1, 5001)), 99.9) == 4995


def test_summary_leaves_rejected_requests_out():
    """A request refused at arrival has no completion time: it must not reach
    the percentiles, the span or the throughput, only the rejected count."""
    R = sv.Result
    res = [R(0, 0.0, 0.010, None), R(1, 0.001, 0.004, None),
           R(2, 0.002, float("nan"), None, rejected=True), R(3, 0.003, 0.012, None)]
    s = sv.summarize(res, lambda rid: 100)
    assert s["completed"] == 3 and s["rejected"] == 1
    assert s["span_s"] == pytest.approx(0.012)
    assert s["requests_per_s"] == pytest.approx(3 / 0.012)
    assert s["gpixel_per_s"] == pytest.approx(300 / 0.012 / 1e9)
    lat = sorted([0.010, 0.003, 0.009])
    assert s["p50_ms"] == pytest.approx(lat[1] * 1e3)
    assert s["p99_ms"] == pytest.approx(lat[2] * 1e3)
    assert all(not math.isnan(v) for v in s.values())
    assert sv.summarize([R(5, 0.0, float("nan"), None, rejected=True)], lambda r: 1) == \
        dict(completed=0, rejected=1)


def test_budget_too_small_rejects_at_arrival():
    """With a budget below one request's bytes the scheduler refuses it at
    offer time; requests that fit still queue and run in FIFO order."""
    big = sv.Request(0, 0.0, 2048, 2048, 3, False)
    small = sv.Request(1, 0.0, 256, 256, 2, True)
    budget = sv.request_bytes(small) * 2
    assert sv.request_bytes(big) > budget
    sch = sv.Scheduler(budget)
    assert sch.offer(big) is False and sch.rejected == [big]
    assert sch.offer(small) is True
    assert [a.req.rid for a in sch.admit(0.0)] == [1]


def test_iteration_pixel_cap_advances_the_oldest_first():
    reqs = [sv.Request(0, 0.0, 1024, 1024, 2, False),     # level inputs 1024^2, 512^2
            sv.Request(1, 0.0, 512, 512, 3, True),        # inverse: 128^2, 256^2, 512^2
            sv.Request(2, 0.0, 2048, 2048, 1, False)]
    assert [sv.level_pixels(reqs[1], k) for k in range(3)] == [128 * 128, 256 * 256, 512 * 512]
    assert [sv.level_pixels(reqs[0], k) for k in range(2)] == [1024 * 1024, 512 * 512]
    sch = sv.Scheduler(1 << 40, max_iteration_pixels=1024 * 1024 + 128 * 128)
    for r in reqs:
        sch.offer(r)
    sch.admit(0.0)
    it = sch.iteration()
    assert [a.req.rid for a in it] == [0, 1]              # request 2 would exceed the cap
    sch.finish_iteration(it)
    it = sch.iteration()
    assert [a.req.rid for a in it] == [0, 1]              # 512^2 + 256^2 leave no room for 2048^2
    done = sch.finish_iteration(it)
    assert [a.req.rid for a in done] == [0]
    it = sch.iteration()
    assert [a.req.rid for a in it] == [1]                 # 512^2 + 2048^2 > cap: oldest only
    sch.finish_iteration(it)
    it = sch.iteration()
    assert [a.req.rid for a in it] == [2]                 # alone it may exceed the cap
    assert sv.Scheduler(1 << 40).max_iteration_pixels is None


def test_request_steps_pair_levels_from_the_finest():
    assert sv.request_steps(5, False, True) == [(1, 2), (3, 4), (5,)]
    assert sv.request_steps(5, True, True) == [(5,), (4, 3), (2, 1)]
    assert sv.request_steps(4, True, True) == [(4, 3), (2, 1)]
    assert sv.request_steps(1, False, True) == [(1,)] == sv.request_steps(1, True, True)
    assert sv.request_steps(3, False, False) == [(1,), (2,), (3,)]
    assert sv.request_steps(3, True, False) == [(3,), (2,), (1,)]
    for L in range(1, 7):
        for inv in (False, True):
            steps = sv.request_steps(L, inv, True)
            assert sorted(j for g in steps for j in g) == list(range(1, L + 1))
            assert len(steps) == (L + 1) // 2


def test_fused_scheduler_finishes_in_half_the_iterations_and_caps_by_finest_level():
    reqs = [sv.Request(0, 0.0, 1024, 1024, 5, False), sv.Request(1, 0.0, 512, 512, 4, True)]
    assert [sv.step_pixels(reqs[0], k, True) for k in range(3)] == [1024 ** 2, 256 ** 2, 64 ** 2]
    assert [sv.step_pixels(reqs[1], k, True) for k in range(2)] == [128 ** 2, 512 ** 2]
    sch = sv.Scheduler(1 << 40, fuse_heads=True)
    for r in reqs:
        assert sch.offer(r)
    sch.admit(0.0)
    finished = {}
    for it in range(1, 10):
        for a in sch.finish_iteration(sch.iteration()):
            finished[a.req.rid] = it
        if sch.idle:
            break
    assert finished == {0: 3, 1: 2}
    capped = sv.Scheduler(1 << 40, max_iteration_pixels=1024 ** 2, fuse_heads=True)
    for r in reqs:
        capped.offer(r)
    capped.admit(0.0)
    assert [a.req.rid for a in capped.iteration()] == [0]      # 1024^2 + 128^2 > cap


def test_head_batch_rejects_bad_pairs_before_any_launch():
    lib = _lib.load()
    F = 0x10000000
    E, U = _lib.ERR_INVALID_ARG, _lib.ERR_UNSUPPORTED

    def job(full, full_dt, ll, ll_dt, bands, w, h):
        j = _lib.LevelJob()
        j.full, j.full_pitch, j.full_dtype = full, w, full_dt
        j.ll, j.ll_pitch, j.ll_dtype = ll, w // 2, ll_dt
        j.hl, j.lh, j.hh = bands, bands + (1 << 20), bands + (2 << 20)
        j.band_pitch, j.band_dtype = w // 2, _lib.F32
        j.width, j.height = w, h
        return j

    mid = F + (1 << 26)
    fine = job(F, _lib.F32, mid, _lib.F32, F + (2 << 26), 64, 64)
    coarse = job(mid, _lib.F32, F + (3 << 26), _lib.F32, F + (4 << 26), 32, 32)

    def call(pair, scheme=0, fn="dwt2_forward_head_batch"):
        arr = (_lib.LevelJob * len(pair))(*pair)
        return getattr(lib, fn)(arr, len(pair) // 2, 0, scheme, None)

    assert lib.dwt2_forward_head_batch(None, 0, 0, 0, None) == 0            # nothing to do
    assert call([fine, coarse], scheme=2) == U                              # LDS ablation
    bad = job(mid, _lib.F32, F + (3 << 26), _lib.F32, F + (4 << 26), 32, 16)
    assert call([fine, bad]) == E                                           # not half size
    other = job(mid + 4096, _lib.F32, F + (3 << 26), _lib.F32, F + (4 << 26), 32, 32)
    assert call([fine, other]) == E                                         # band not shared
    half = job(F, _lib.F32, mid, _lib.F16, F + (2 << 26), 64, 64)
    assert call([half, coarse]) == E                                        # band not FP32
    clash = job(mid, _lib.F32, F + (2 << 26), _lib.F32, F + (4 << 26), 32, 32)
    assert call([fine, clash]) == E                   # forward: coarse ll on fine hl, both written
    out_on_band = job(F + (4 << 26), _lib.F32, mid, _lib.F32, F + (2 << 26), 64, 64)
    assert call([out_on_band, coarse], fn="dwt2_inverse_head_batch") == E   # output on a read band


@pytest.mark.parametrize("levels", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("inverse", [False, True])
def test_fused_layout_never_writes_what_a_step_reads(levels, inverse):
    torch = pytest.importorskip("torch")
    W, H = 512, 320
    src = torch.zeros(H, W, dtype=torch.float16)
    out = torch.zeros_like(src)
    n0 = (W // 2) * (H // 2) if levels > 1 else 1
    n1 = (W // 4) * (H // 4) if levels > 2 else 1
    ws0, ws1 = torch.zeros(n0), torch.zeros(n1)
    jobs = sv.level_jobs(src, out, ws0, ws1, levels, inverse, fuse_heads=True)
    index = {(levels - k if inverse else k + 1): k for k in range(levels)}
    bufs = [(ws0.data_ptr(), 4 * n0), (ws1.data_ptr(), 4 * n1)]

    def span(ptr, rows, pitch, es):
        return ptr, ptr + rows * pitch * es

    def inside_ws(lo, hi):
        return any(b <= lo and hi <= b + n for b, n in bufs)

    def apart(a, b):
        return a[1] <= b[0] or b[1] <= a[0]

    for j in range(1, levels):                     # every FP32 band fits its buffer
        jb = jobs[index[j]]
        assert inside_ws(*span(jb.ll, jb.height // 2, jb.ll_pitch, 4))
    for g in sv.request_steps(levels, inverse, True):
        if len(g) == 1:
            continue
        fine, coarse = jobs[index[min(g)]], jobs[index[max(g)]]
        assert fine.ll == coarse.full and fine.ll_pitch == coarse.full_pitch
        first = span(fine.full, fine.height, fine.full_pitch, 2 if min(g) == 1 else 4)
        last = span(coarse.ll, coarse.height // 2, coarse.ll_pitch,
                    2 if max(g) == levels else 4)
        assert apart(first, last)                 # the pair's input and output
        mid = span(fine.ll, fine.height // 2, fine.ll_pitch, 4)
        assert apart(mid, first) and apart(mid, last)


def test_admitted_step_bookkeeping_matches_request_steps():
    for L in range(1, 8):
        for inv in (False, True):
            for fuse in (False, True):
                req = sv.Request(0, 0.0, 1 << 9, 3 << 8, L, inv)
                a = sv._Active(req, 0, 0.0, fuse)
                steps = sv.request_steps(L, inv, fuse)
                assert a.steps == [len(g) for g in steps]
                assert a.step_px == [sv.step_pixels(req, k, fuse) for k in range(len(steps))]
