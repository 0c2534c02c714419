"""Serving loop: continuous batching of independent DWT requests on one GPU.

Each request is one image (forward) or one Mallat pyramid (inverse) with its
own level count. The loop works in iterations: an iteration advances every
active request by one step, enqueued as a few batched launches grouped by
size class and storage types inside the library. A step is one level
(dwt2_forward_level_batch / dwt2_inverse_level_batch) or, with fused heads
(the default), two consecutive levels in one head launch
(dwt2_forward_head_batch / dwt2_inverse_head_batch), paired from the finest
level up, which keeps the band between them on chip and halves the steps. New
arrivals join at the next iteration and finished requests leave, so large and
small requests share the device without a small one waiting for a large one
to finish all its levels.

Admission is first-come first-served under an HBM budget: a request holds its
input, its output pyramid and its FP32 intermediate low-low buffers from
admission until the client releases the result. A request that can never fit
is rejected at arrival.

``Scheduler`` is the host-side policy (no GPU, testable with a simulated
clock); ``Server`` allocates buffers with PyTorch, builds the per-level job
descriptors once at admission and drives the library on one HIP stream.
Latency is measured from the request's arrival to the GPU timestamp of the
iteration that finished it.
"""
from __future__ import annotations

import collections
import ctypes
import dataclasses
import fractions
import gc
import math
import time

from . import _lib
from . import _scheme, _stream_ptr, _wavelet, load

_STORAGE_BYTES = {_lib.F32: 4, _lib.F16: 2, _lib.BF16: 2}


@dataclasses.dataclass
class Request:
    """A transform asked for by a client. `width` x `height` must be divisible
    by 2**levels."""
    rid: int
    arrival_s: float
    width: int
    height: int
    levels: int
    inverse: bool


def workspace_bytes(width: int, height: int, levels: int) -> int:
    """FP32 intermediate low-low buffers of one request (two ping-pong
    buffers, the larger a quarter of the image)."""
    if levels <= 1:
        return 0
    n = (width // 2) * (height // 2)
    if levels >= 3:
        n += (width // 4) * (height // 4)
    return 4 * n


def request_bytes(req: Request, dtype: int = _lib.F16) -> int:
    """HBM held by an admitted request: input + output in the storage type and
    the FP32 intermediates."""
    px = req.width * req.height
    return 2 * px * _STORAGE_BYTES[dtype] + workspace_bytes(req.width, req.height, req.levels)


class _Active:
    __slots__ = ("req", "bytes", "next_level", "t_admit", "payload", "steps", "step_px")

    def __init__(self, req, nbytes, t_admit, fuse_heads=False):
        self.req = req
        self.bytes = nbytes
        self.next_level = 0          # steps already enqueued (levels without fused heads)
        self.t_admit = t_admit
        self.payload = None
        # per step, the number of levels it runs and the input pixels of its
        # finest level (request_steps, computed inline: this runs per admission)
        L, W, H = req.levels, req.width, req.height
        sizes = [2] * (L // 2) + [1] * (L % 2) if fuse_heads else [1] * L
        if req.inverse:
            sizes.reverse()
        self.steps = sizes
        px, top = [], (L if req.inverse else 1)
        for n in sizes:
            j = top - n + 1 if req.inverse else top      # finest level of the step
            px.append((W >> (j - 1)) * (H >> (j - 1)))
            top = top - n if req.inverse else top + n
        self.step_px = px


def request_steps(levels: int, inverse: bool, fuse_heads: bool = False):
    """The launches of one request in execution order, each a tuple of the
    levels it runs: one level, or with fuse_heads two consecutive levels in
    one head launch, paired from the finest level up ((1, 2), (3, 4), ...; an
    odd top level runs alone). A forward runs finest first; an inverse runs
    coarsest first, a pair as (j + 1, j)."""
    groups, j = [], 1
    while j <= levels:
        if fuse_heads and j + 1 <= levels:
            groups.append((j, j + 1))
            j += 2
        else:
            groups.append((j,))
            j += 1
    if inverse:
        return [tuple(reversed(g)) for g in reversed(groups)]
    return groups


def step_pixels(req: Request, step: int, fuse_heads: bool = False) -> int:
    """Input pixels of the finest level that a request's step-th launch
    (0-based, execution order) runs: the measure of its work."""
    j = min(request_steps(req.levels, req.inverse, fuse_heads)[step])
    return (req.width >> (j - 1)) * (req.height >> (j - 1))


def level_pixels(req: Request, level: int) -> int:
    """Input pixels of a request's level-th launch (0-based, in execution
    order: the forward starts at the full image, the inverse at the coarsest
    level)."""
    j = req.levels - level if req.inverse else level + 1
    return (req.width >> (j - 1)) * (req.height >> (j - 1))


class Scheduler:
    """FIFO admission under a byte budget and a cap on active requests;
    level-synchronous iterations, optionally capped in work.

    offer(req)        queue an arrived request (False if it can never fit)
    admit(now)        move queue heads into the active set while they fit
    iteration()       the active requests to advance by one step now: all of
                      them, or with max_iteration_pixels the oldest ones whose
                      steps' finest level inputs add up to at most that many
                      pixels (always at least the oldest), so that one
                      iteration's device time stays bounded however many
                      requests are admitted
    finish_iteration  advance them; returns those that have enqueued their
                      last step (their bytes stay held until release())

    A step is one level, or with fuse_heads a pair of levels (request_steps).
    release(a)        return a finished request's bytes to the budget
    """

    def __init__(self, budget_bytes: int, max_active: int = 1 << 30, bytes_fn=request_bytes,
                 max_iteration_pixels: int | None = None, fuse_heads: bool = False):
        self.budget = int(budget_bytes)
        self.fuse_heads = bool(fuse_heads)
        self.max_active = int(max_active)
        self.max_iteration_pixels = max_iteration_pixels
        self.bytes_fn = bytes_fn
        self.queue = collections.deque()
        self.active = []
        self.used = 0
        self.peak_used = 0
        self.rejected = []

    def offer(self, req: Request) -> bool:
        if self.bytes_fn(req) > self.budget:
            self.rejected.append(req)
            return False
        self.queue.append(req)
        return True

    def admit(self, now: float):
        admitted = []
        while self.queue and len(self.active) < self.max_active:
            req = self.queue[0]
            nb = self.bytes_fn(req)
            if self.used + nb > self.budget:
                break                          # strict FIFO: no overtaking
            self.queue.popleft()
            a = _Active(req, nb, now, self.fuse_heads)
            self.active.append(a)
            self.used += nb
            admitted.append(a)
        self.peak_used = max(self.peak_used, self.used)
        return admitted

    def iteration(self):
        if self.max_iteration_pixels is None:
            return list(self.active)
        out, px = [], 0
        for a in self.active:                  # admission order: oldest first
            p = a.step_px[a.next_level]
            if out and px + p > self.max_iteration_pixels:
                break
            out.append(a)
            px += p
        return out

    def finish_iteration(self, advanced):
        done = []
        for a in advanced:
            a.next_level += 1
            if a.next_level == len(a.step_px):
                done.append(a)
        if done:
            ids = {id(a) for a in done}
            self.active = [a for a in self.active if id(a) not in ids]
        return done

    def release(self, a: _Active):
        self.used -= a.bytes

    @property
    def idle(self) -> bool:
        return not self.queue and not self.active


# ---------------------------------------------------------------------------
# GPU side


def _job(full, ll, hl, lh, hh, width, height, dtcode):
    """A job from tensors (hl, lh and hh share one row pitch)."""
    j = _lib.LevelJob()
    j.full, j.full_pitch, j.full_dtype = full.data_ptr(), full.stride(0), dtcode(full)
    j.ll, j.ll_pitch, j.ll_dtype = ll.data_ptr(), ll.stride(0), dtcode(ll)
    j.hl, j.lh, j.hh = hl.data_ptr(), lh.data_ptr(), hh.data_ptr()
    j.band_pitch, j.band_dtype = hl.stride(0), dtcode(hl)
    j.width, j.height = width, height
    return j


def ll_slots(width: int, height: int, levels: int, fuse_heads: bool = False):
    """Where each intermediate low-low band LL_k (1 <= k < levels, the output
    of level k's forward) lives: k -> (buffer 0 or 1, offset in floats).

    One level per step: LL_k alternates between ws0 and ws1 at offset 0 (a
    level reads one and writes the other). With fused heads (request_steps),
    the bands that steps store, LL_2, LL_4, ..., alternate between ws1 and ws0,
    so that a step never writes the buffer it reads; the band inside a pair,
    LL_k for odd k, is never accessed but needs a place of its own: ws0 at 0
    for LL_1, else ws0 just past the stored band there (LL_(k-1) is at most
    (W >> (k-1)) * (H >> (k-1)) floats). ws0 holds (W/2)(H/2) floats and ws1
    (W/4)(H/4), which is enough for every slot."""
    slots = {}
    for k in range(1, levels):
        if not fuse_heads:
            slots[k] = ((k - 1) % 2, 0)
        elif k % 2 == 0:
            slots[k] = (1 if (k // 2) % 2 == 1 else 0, 0)
        elif k == 1:
            slots[k] = (0, 0)
        else:
            slots[k] = (0, (width >> (k - 1)) * (height >> (k - 1)))
    return slots


def level_jobs(src, out, ws0, ws1, levels, inverse, fuse_heads=False):
    """Per-level job descriptors of one request, in execution order.

    Forward: level j reads the image (j = 1) or the previous low-low band and
    writes its detail bands into the Mallat quadrants of `out` and its
    low-low band to an FP32 buffer (or to the top-left of `out` at the last
    level). Inverse: levels L..1 mirror that, reading the pyramid `src` and
    writing the image to `out`. ws0 holds a quarter of the image, ws1 a
    sixteenth; the FP32 bands take the places ll_slots gives (with
    fuse_heads, a layout in which every pair of request_steps can run as one
    head launch). Pointers are computed directly (this runs once per admitted
    request).
    """
    from . import _dtype_code
    H, W = src.shape
    P = src.stride(0)
    if out.stride(0) != P or out.shape != src.shape or out.dtype != src.dtype:
        raise ValueError("src and out must share shape, dtype and row pitch")
    dt = _dtype_code(src)
    e = src.element_size()
    pyr = (src if inverse else out).data_ptr()
    img = (out if inverse else src).data_ptr()
    ws = (ws0.data_ptr(), ws1.data_ptr())
    slots = ll_slots(W, H, levels, fuse_heads)

    def band(k):                     # address of LL_k
        b, off = slots[k]
        return ws[b] + 4 * off

    jobs = (_lib.LevelJob * levels)()
    order = range(levels, 0, -1) if inverse else range(1, levels + 1)
    for k, j in enumerate(order):
        h, w = H >> (j - 1), W >> (j - 1)
        h2, w2 = h // 2, w // 2
        job = jobs[k]
        if j == 1:
            job.full, job.full_pitch, job.full_dtype = img, P, dt
        else:
            job.full, job.full_pitch, job.full_dtype = band(j - 1), w, _lib.F32
        if j == levels:
            job.ll, job.ll_pitch, job.ll_dtype = pyr, P, dt
        else:
            job.ll, job.ll_pitch, job.ll_dtype = band(j), w2, _lib.F32
        job.hl = pyr + e * w2
        job.lh = pyr + e * h2 * P
        job.hh = pyr + e * (h2 * P + w2)
        job.band_pitch, job.band_dtype = P, dt
        job.width, job.height = w, h
    return jobs


@dataclasses.dataclass
class Result:
    rid: int
    arrival_s: float
    done_s: float          # GPU completion time, same clock as arrival_s (NaN if rejected)
    output: object         # the output tensor (None once released by the server)
    rejected: bool = False  # refused at arrival: it can never fit the admission budget

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


def summarize(results, pixels_of) -> dict:
    """Throughput and latency of one served trace. Rejected requests count
    only in `rejected`: they have no completion time and take no part in the
    latency percentiles, the span or the throughput. pixels_of(rid) gives a
    request's image pixels."""
    done = [r for r in results if not r.rejected]
    out = dict(completed=len(done), rejected=len(results) - len(done))
    if not done:
        return out
    lat = [r.latency_s for r in done]
    span = max(r.done_s for r in done) - min(r.arrival_s for r in done)
    px = sum(pixels_of(r.rid) for r in done)
    out.update(span_s=span, requests_per_s=len(done) / span, gpixel_per_s=px / span / 1e9,
               p50_ms=percentile(lat, 50) * 1e3, p99_ms=percentile(lat, 99) * 1e3,
               p999_ms=percentile(lat, 99.9) * 1e3)
    return out


class Server:
    """Runs a request trace through the continuous-batching loop on the
    current HIP device.

    inputs: rid -> 2-D GPU tensor (the image, or the pyramid of an inverse
    request), resident before the request arrives. keep_outputs keeps every
    result's output tensor (tests); otherwise results are released as soon as
    the iteration that finished them is observed complete.
    """

    def __init__(self, budget_bytes=64 << 30, max_active=1 << 30, wavelet="cdf97",
                 scheme="nonseparable", dtype="f16", class_tiles=None, max_inflight=2,
                 max_iteration_pixels=None, fuse_heads=True):
        self.dtype = {"f32": _lib.F32, "f16": _lib.F16, "bf16": _lib.BF16}[dtype]
        self.fuse_heads = bool(fuse_heads)
        self.sched = Scheduler(budget_bytes, max_active,
                               bytes_fn=lambda r: request_bytes(r, self.dtype),
                               max_iteration_pixels=max_iteration_pixels,
                               fuse_heads=self.fuse_heads)
        self.wavelet = _wavelet(wavelet)
        self.scheme = _scheme(scheme)
        self.class_tiles = (None if class_tiles is None else
                            (ctypes.c_int32 * _lib.SIZE_CLASSES)(*class_tiles))
        self.max_inflight = max_inflight
        self.iterations = 0
        self.launch_calls = 0
        self.busy_s = 0.0           # summed device time of the iterations (see run)

    def _allocate(self, a, inputs, torch):
        req = a.req
        src = inputs[req.rid]
        if src.shape != (req.height, req.width):
            raise ValueError(f"request {req.rid}: input shape {tuple(src.shape)}")
        out = torch.empty_like(src)
        n0 = (req.width // 2) * (req.height // 2) if req.levels > 1 else 1
        n1 = (req.width // 4) * (req.height // 4) if req.levels > 2 else 1
        ws0 = torch.empty(n0, dtype=torch.float32, device=src.device)
        ws1 = torch.empty(n1, dtype=torch.float32, device=src.device)
        jobs = level_jobs(src, out, ws0, ws1, req.levels, req.inverse, self.fuse_heads)
        # first job (execution order) of each step
        first, k = [], 0
        for n in a.steps:
            first.append(k)
            k += n
        a.payload = {"out": out, "ws": (ws0, ws1), "jobs": jobs, "first": first}

    def _enqueue(self, advanced, stream):
        lib = load()
        calls = {(inv, n): [] for inv in (False, True) for n in (1, 2)}
        for a in advanced:
            jobs, k = a.payload["jobs"], a.payload["first"][a.next_level]
            n, inv = a.steps[a.next_level], a.req.inverse
            if n == 1:
                calls[(inv, 1)].append(jobs[k])
            else:                        # a head pair as (finer, coarser) level
                calls[(inv, 2)] += (jobs[k + 1], jobs[k]) if inv else (jobs[k], jobs[k + 1])
        fns = {(False, 1): ("dwt2_forward_level_batch", True),
               (True, 1): ("dwt2_inverse_level_batch", True),
               (False, 2): ("dwt2_forward_head_batch", False),
               (True, 2): ("dwt2_inverse_head_batch", False)}
        for key, jobs in calls.items():
            if not jobs:
                continue
            name, tiles = fns[key]
            arr = (_lib.LevelJob * len(jobs))(*jobs)
            n = len(jobs) // key[1]
            args = (arr, n, self.wavelet, self.scheme) + ((self.class_tiles,) if tiles else ())
            _lib.check(getattr(lib, name)(*args, stream), name)
            self.launch_calls += 1

    def run(self, requests, inputs, keep_outputs=False, realtime=True):
        """Serve `requests` (sorted by arrival). With realtime=False every
        request is offered at time zero (saturation). Returns the results in
        completion order."""
        import torch
        from . import _dtype_code
        for r in requests:
            if _dtype_code(inputs[r.rid]) != self.dtype:
                raise ValueError(f"request {r.rid}: input dtype differs from the server's")
        stream = torch.cuda.current_stream()
        sptr = _stream_ptr(stream)
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival_s))
        inflight = collections.deque()          # (start event, end event, finished actives)
        results = []
        start = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        start.record(stream)

        def retire(ev0, ev, done):
            ms = start.elapsed_time(ev)
            # an iteration's device time: from the stream reaching its launches
            # to their end (when the device was idle before it, this includes
            # the host's launch latency: an upper bound)
            self.busy_s += ev0.elapsed_time(ev) / 1e3
            for a in done:
                out = a.payload["out"]
                results.append(Result(a.req.rid, a.req.arrival_s if realtime else 0.0,
                                       ms / 1e3, out if keep_outputs else None))
                a.payload = None
                self.sched.release(a)

        # The loop's objects are freed by reference counting; the cyclic
        # collector is paused for the run, since its passes over the many live
        # objects (requests, buffers, events) stall iterations by tens of ms.
        gc_was_enabled = gc.isenabled()
        gc.disable()
        try:
            while pending or not self.sched.idle or inflight:
                now = time.perf_counter() - t0
                while pending and (not realtime or pending[0].arrival_s <= now):
                    r = pending.popleft()
                    if not self.sched.offer(r):            # can never fit the budget
                        results.append(Result(r.rid, r.arrival_s, float("nan"), None,
                                              rejected=True))
                for a in self.sched.admit(now):
                    self._allocate(a, inputs, torch)
                advanced = self.sched.iteration()
                if advanced:
                    ev0 = torch.cuda.Event(enable_timing=True)
                    ev0.record(stream)
                    self._enqueue(advanced, sptr)
                    done = self.sched.finish_iteration(advanced)
                    ev = torch.cuda.Event(enable_timing=True)
                    ev.record(stream)
                    inflight.append((ev0, ev, done))
                    self.iterations += 1
                # observe completions; keep at most max_inflight iterations queued
                while inflight and (len(inflight) > self.max_inflight or inflight[0][1].query()
                                    or (not advanced and not pending)):
                    ev0, ev, done = inflight.popleft()
                    ev.synchronize()
                    retire(ev0, ev, done)
                if not advanced and not inflight and pending and realtime:
                    wait = pending[0].arrival_s - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 1e-3))
        finally:
            if gc_was_enabled:
                gc.enable()
        return results


def percentile(values, q):
    """Nearest-rank percentile (q in 0..100) of a non-empty list: the
    ceil(q/100 * n)-th smallest value."""
    v = sorted(values)
    rank = math.ceil(fractions.Fraction(str(q)) * len(v) / 100)   # exact for q = 99.9
    return v[max(0, min(len(v) - 1, rank - 1))]
