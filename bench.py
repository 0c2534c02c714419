#!/usr/bin/env python3
"""Benchmark of the 2-D DWT hot path on one MI355X.

A step is one forward plus one inverse L-level transform of one image that is
already resident in HBM. The default workload is the headline one: a
4096 x 4096 FP32 image (sum of random sinusoids plus noise), CDF 9/7, five
levels, non-separable lifting. Steps rotate over several buffer sets, so
many that the images of all sets together exceed twice the 256 MB Infinity
Cache: each step, and each launch of the per-level timing loops, reads its
input from HBM rather than from the cache.

Prints one JSON line with the throughput in Gpixel/s (original-image pixels
per second of forward+inverse), the roofline of the dominant kernel
(level-1 launch, HBM-bound; also as a fraction of the runtime's measured
device-copy bandwidth), the median and p10 / p90 of single steps, the same
steps with a warm Infinity Cache, the separable-lifting kernel measured the
same way, both schemes with every neighbour exchange through LDS (the
barrier ablation), the serving half of the metric (p50/p99 latency of the
mixed FP16 request stream at 0.8 of its saturation rate), and the FP64
oracle timed on the host cores (all cores and one).

Other workloads: --workload batch (256 uneven images, batched launches in a
graph) and --workload serve (the full serving sweep); --size, --levels,
--wavelet and --dtype select the other image configurations.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = ("Gpixel/s fwd+inv CDF 9/7 DWT at 4096², 5 levels (% HBM peak); "
          "serving p50/p99")
# Traffic counters are valid for the kernel code they were taken with (these
# sources) and the tile geometry named in their key.
KERNEL_SOURCES = ("dwt2_device.hpp", "dwt2_kernels.hpp", "dwt2_head.hpp", "dwt2_tail.hpp")


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for n in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1705_08266_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


INFINITY_CACHE_BYTES = 256 << 20
STEP_SAMPLES = 50   # individually timed steps for the median and p10 / p90


def buffer_sets(args, W, H) -> int:
    """Rotating buffer sets: --sets, else enough that the images of all sets
    together hold at least twice the Infinity Cache (4..64 sets)."""
    if args.sets:
        return args.sets
    es = {"f32": 4, "f16": 2, "bf16": 2}[args.dtype]
    need = -(-2 * INFINITY_CACHE_BYTES // (W * H * es))
    return min(64, max(4, need))


def level_bytes(W, H, levels, es_store):
    """Algorithmic HBM bytes of each forward level launch (the inverse level is
    symmetric): read the level input once, write its four bands once. The
    user-visible image and bands use the storage size; intermediate LL is FP32."""
    out = []
    for j in range(1, levels + 1):
        w, h = W >> (j - 1), H >> (j - 1)
        px = w * h
        in_es = es_store if j == 1 else 4
        ll_es = es_store if j == levels else 4
        out.append(px * in_es + (px // 4) * (3 * es_store + ll_es))
    return out


def launch_units(levels, fused, head):
    """The launches of one direction of the chain, finest first: (kind, first
    level, number of levels) with kind "head" (levels 1 and 2 fused), "level"
    (one level) or "tail" (the last `fused` levels fused)."""
    units = []
    j = 1
    if head:
        units.append(("head", 1, 2))
        j = 3
    k = levels - fused + 1 if fused >= 2 else levels + 1
    while j < k:
        units.append(("level", j, 1))
        j += 1
    if fused >= 2:
        units.append(("tail", k, fused))
    return units


def unit_bytes(W, H, levels, es_store, unit):
    """Algorithmic bytes of one forward launch (the inverse is symmetric): one
    read of its first level's input, one write of every level's detail bands
    and of its last level's LL. Low-low bands between its levels stay on chip;
    the image and bands use the storage size, intermediate LL is FP32."""
    _, k, n = unit
    w, h = W >> (k - 1), H >> (k - 1)
    b = w * h * (es_store if k == 1 else 4)
    for j in range(k, k + n):
        px = (W >> (j - 1)) * (H >> (j - 1))
        b += (px // 4) * 3 * es_store
    last = k + n - 1
    b += (W >> last) * (H >> last) * (es_store if last == levels else 4)
    return b


def executed_bytes(W, H, levels, es_store, fused, head=False):
    """Algorithmic bytes per direction of the launches actually made."""
    return sum(unit_bytes(W, H, levels, es_store, u)
               for u in launch_units(levels, fused, head))


def make_image(W, H, kind, seed):
    import synthetic
    if kind == "sinusoid":
        return synthetic.sinusoid_image(H, W, seed=seed)
    return synthetic.uniform_image(H, W, seed=seed)


def run_gpu(args, x_np, scheme):
    """Time K steps (graph replays of forward + inverse) and, separately, the
    level-1 kernels back to back with events; returns timings and outputs."""
    import torch
    import paper_1705_08266_amd as dwt
    from paper_1705_08266_amd import _lib

    tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[args.dtype]
    H, W = x_np.shape
    L = args.levels
    dev = torch.device("cuda:0")
    x0 = torch.from_numpy(x_np).to(dev).to(tdt)
    sets = []
    for s in range(buffer_sets(args, W, H)):
        src = x0.clone()
        coef = torch.empty_like(src)
        rec = torch.empty_like(src)
        ws = dwt.make_workspace(W, H, L, dev)
        sets.append((src, coef, rec, ws))

    # --fuse off: one launch per level (the library's per-level choice)
    chain_tiles = [dwt.default_tile(W >> j, H >> j) for j in range(L)] if args.fuse == "off" \
        else None

    def step(k):
        src, coef, rec, ws = sets[k % len(sets)]
        dwt.forward(src, args.wavelet, L, scheme, out=coef, workspace=ws, tiles=chain_tiles)
        dwt.inverse(coef, args.wavelet, L, scheme, out=rec, workspace=ws, tiles=chain_tiles)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    eager_coef = sets[0][1].clone()
    eager_rec = sets[0][2].clone()

    # one captured graph per buffer set (the whole L-level forward and inverse
    # chain), and one graph that holds a step on every buffer set
    graphs = []
    for k in range(len(sets)):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step(k)
        graphs.append(g)
    multi = torch.cuda.CUDAGraph()
    with torch.cuda.graph(multi):
        for k in range(len(sets)):
            step(k)
    for k in range(2 * len(sets)):
        graphs[k % len(sets)].replay()
    multi.replay()
    torch.cuda.synchronize()

    # The timed steps: host calls of the library by default, as a caller makes
    # them (a graph launch costs a few microseconds of its own on this stack);
    # --graph replays the per-step graphs instead.
    def run_step(k):
        if args.graph:
            graphs[k % len(graphs)].replay()
        else:
            step(k)

    stream = torch.cuda.current_stream()
    K = args.steps

    def timed_ms(fn, n):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        for k in range(n):
            fn(k)
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    w0 = time.perf_counter()
    total_ms = timed_ms(run_step, K)
    wall = time.perf_counter() - w0

    # the same K steps as graph replays: one graph per step, and graphs of
    # len(sets) steps each (the last writes every buffer set)
    graph_ms = dict(per_step=timed_ms(lambda k: graphs[k % len(graphs)].replay(), K) / K,
                    multi_step=timed_ms(lambda k: multi.replay(), max(1, K // len(sets)))
                    / (max(1, K // len(sets)) * len(sets)),
                    steps_per_graph=len(sets))
    replay_matches = bool(torch.equal(sets[0][1], eager_coef) and torch.equal(sets[0][2], eager_rec))

    # Spread of single steps: each bracketed by its own events (cold buffers,
    # rotating as above).
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
             for _ in range(STEP_SAMPLES)]
    for k, (a, b) in enumerate(pairs):
        a.record(stream)
        run_step(k)
        b.record(stream)
    torch.cuda.synchronize()
    step_ms = sorted(a.elapsed_time(b) for a, b in pairs)

    # Warm cache: the same buffer set every step, so the image and its
    # coefficients stay in the Infinity Cache.
    run_step(0)
    warm_ms = timed_ms(lambda k: run_step(0), K) / K

    # The same K steps with consecutive steps (independent buffer sets) on two
    # streams, so that one chain's launch gaps overlap the other's kernels.
    concurrent_ms = None
    if len(graphs) >= 2:
        side = [torch.cuda.Stream(), torch.cuda.Stream()]   # default priority
        for _ in range(2):
            c0 = torch.cuda.Event(enable_timing=True)
            c1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            c0.record(stream)
            for st in side:
                st.wait_event(c0)
            for k in range(K):
                with torch.cuda.stream(side[k % 2]):
                    graphs[k % len(graphs)].replay()
            for st in side:
                stream.wait_stream(st)
            c1.record(stream)
            torch.cuda.synchronize()
            concurrent_ms = c0.elapsed_time(c1)

    # per-launch kernel durations: each launch of the chain repeated back to
    # back, bracketed by events on the launch stream, buffers rotating
    R = 40
    fwd_ms, inv_ms = [], []
    # the exchange-ablation schemes never fuse levels
    lds = scheme.endswith("_lds")
    fused = dwt.fused_levels(W, H, L) if args.fuse == "auto" and not lds else 0
    head = args.fuse == "auto" and not lds and dwt.head_levels(W, H, L) == 2
    units = launch_units(L, fused, head)
    for kind, j, nlev in units:
        w, h = W >> (j - 1), H >> (j - 1)
        for direction in ("forward", "inverse"):
            def once(k):
                # the same kernel instantiations as the chain: intermediate LL
                # bands live in the FP32 workspace, split in two regions
                src, coef, rec, ws = sets[k % len(sets)]
                big = (W // 2) * (H // 2)
                hl, lh, hh = coef[:h // 2, w // 2:w], coef[h // 2:h, :w // 2], coef[h // 2:h, w // 2:w]
                if j == L:
                    ll = coef[:h // 2, :w // 2]
                elif j == 1:
                    ll = ws[:big].view(H // 2, W // 2)
                else:
                    ll = ws[big:big + (w // 2) * (h // 2)].view(h // 2, w // 2)
                if j == 1:
                    img = src if direction == "forward" else rec
                else:
                    img = ws[:w * h].view(h, w)
                if kind == "head":
                    # levels 1 and 2 of the full image: the bands go to their
                    # places in coef; the level-2 LL to coef's corner instead
                    # of the workspace (the same FP32 kernel)
                    if direction == "forward":
                        dwt.forward(src, args.wavelet, 2, scheme, out=coef, workspace=ws,
                                    tiles=[_lib.TILE_HEAD] * 2)
                    else:
                        dwt.inverse(coef, args.wavelet, 2, scheme, out=rec, workspace=ws,
                                    tiles=[_lib.TILE_HEAD] * 2)
                elif kind == "tail":
                    # the fused launch of levels j..L on the chain's buffers:
                    # the level-j input in the workspace, the bands in coef
                    sub = coef[:h, :w]
                    if direction == "forward":
                        dwt.forward(img, args.wavelet, nlev, scheme, out=sub, workspace=tws,
                                    tiles=[_lib.TILE_TAIL] * nlev)
                    else:
                        dwt.inverse(sub, args.wavelet, nlev, scheme, out=img, workspace=tws,
                                    tiles=[_lib.TILE_TAIL] * nlev)
                elif direction == "forward":
                    dwt.forward_level(img, ll, hl, lh, hh, args.wavelet, scheme)
                elif j == 1:
                    # the chain's last launch is the finest level of the
                    # multi-level inverse, which streams a large image past
                    # the caches; a one-level inverse makes the same launch
                    dwt.inverse(coef, args.wavelet, 1, scheme, out=rec, workspace=ws)
                else:
                    dwt.inverse_level(ll, hl, lh, hh, img, args.wavelet, scheme)
            if kind == "tail" and args.dtype != "f32" and j > 1:
                # a 16-bit chain's tail reads an FP32 LL; a standalone call of
                # the same storage type is a different kernel
                (fwd_ms if direction == "forward" else inv_ms).append(None)
                continue
            # (a 16-bit chain's head writes an FP32 level-2 LL; its stand-in,
            # the two-level call, writes that band in the storage type)
            if kind == "tail":
                tws = dwt.make_workspace(w, h, nlev, dev)
            for k in range(5):
                once(k)
            # R launches captured in one graph, so host launch overhead does
            # not stretch the small levels; buffers rotate as in the chain
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                for k in range(R):
                    once(k)
            g.replay()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            g.replay()
            e1.record(stream)
            torch.cuda.synchronize()
            del g
            (fwd_ms if direction == "forward" else inv_ms).append(e0.elapsed_time(e1) / R)

    out = dict(total_ms=total_ms, wall_s=wall, fwd_level_ms=fwd_ms, inv_level_ms=inv_ms,
               concurrent_ms=concurrent_ms, step_ms=step_ms, warm_ms=warm_ms,
               units=units, fused_levels=list(range(L - fused + 1, L + 1)) if fused else [],
               head=head,
               coef=eager_coef.float().cpu().numpy(), rec=eager_rec.float().cpu().numpy(),
               stored=sets[0][0].float().cpu().numpy(),
               replay_matches_eager=replay_matches, graph=args.graph, graph_ms=graph_ms)
    del sets, graphs
    torch.cuda.empty_cache()
    return out


AB_STEPS = 200     # single steps per scheme in the interleaved comparison
AB_ROUNDS = 10     # alternations of the per-launch timing loops


def ab_schemes(args, x_np):
    """Non-separable against separable lifting, interleaved in one process on
    the same buffers: single steps (host calls, as in the timed loop) alternate
    between the two schemes (the order swapping every step) for AB_STEPS steps each, and the
    per-launch timing loops (20 back-to-back launches of each chain launch)
    alternate AB_ROUNDS times. Returns medians and p10 / p90 of both."""
    import numpy as np
    import torch
    import paper_1705_08266_amd as dwt
    from paper_1705_08266_amd import _lib

    tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[args.dtype]
    H, W = x_np.shape
    L = args.levels
    dev = torch.device("cuda:0")
    x0 = torch.from_numpy(x_np).to(dev).to(tdt)
    sets = [(x0.clone(), torch.empty_like(x0), torch.empty_like(x0),
             dwt.make_workspace(W, H, L, dev)) for _ in range(buffer_sets(args, W, H))]
    schemes = ("nonseparable", "separable")
    stream = torch.cuda.current_stream()

    def step(k, sch):
        src, coef, rec, ws = sets[k % len(sets)]
        dwt.forward(src, args.wavelet, L, sch, out=coef, workspace=ws)
        dwt.inverse(coef, args.wavelet, L, sch, out=rec, workspace=ws)

    for k in range(2 * len(sets)):
        for sch in schemes:
            step(k, sch)
    torch.cuda.synchronize()
    ev = {sch: [] for sch in schemes}
    for k in range(AB_STEPS):
        order = schemes if k % 2 == 0 else schemes[::-1]
        for sch in order:
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            step(k, sch)
            b.record(stream)
            ev[sch].append((a, b))
    torch.cuda.synchronize()
    step_ms = {sch: np.array([a.elapsed_time(b) for a, b in ev[sch]]) for sch in schemes}

    # per-launch loops: the chain's launches (head / levels / tail), 20 each
    fused = dwt.fused_levels(W, H, L)
    units = launch_units(L, fused, dwt.head_levels(W, H, L) == 2)

    def launch(unit, direction, k, sch):
        kind, j, n = unit
        src, coef, rec, ws = sets[k % len(sets)]
        w, h = W >> (j - 1), H >> (j - 1)
        if kind == "level" and j > 1:
            img = ws[:w * h].view(h, w)
            if direction == "forward":
                dwt.forward(img, args.wavelet, 1, sch, out=coef[:h, :w])
            else:
                dwt.inverse(coef[:h, :w], args.wavelet, 1, sch, out=img)
            return
        if kind == "tail" and j > 1:
            img = ws[:w * h].view(h, w)
            tws = tail_ws[unit]
            if direction == "forward":
                dwt.forward(img, args.wavelet, n, sch, out=coef[:h, :w], workspace=tws,
                            tiles=[_lib.TILE_TAIL] * n)
            else:
                dwt.inverse(coef[:h, :w], args.wavelet, n, sch, out=img, workspace=tws,
                            tiles=[_lib.TILE_TAIL] * n)
            return
        tiles = [_lib.TILE_HEAD] * 2 if kind == "head" else \
            ([_lib.TILE_TAIL] * n if kind == "tail" else None)
        if direction == "forward":
            dwt.forward(src, args.wavelet, n, sch, out=coef, workspace=ws, tiles=tiles)
        else:
            dwt.inverse(coef, args.wavelet, n, sch, out=rec, workspace=ws, tiles=tiles)

    # the stand-in launches match the chain's kernels for FP32 storage only (a
    # 16-bit chain keeps an FP32 low-low band on one side of its launches)
    if args.dtype != "f32":
        units = []
    tail_ws = {u: dwt.make_workspace(W >> (u[1] - 1), H >> (u[1] - 1), u[2], dev)
               for u in units if u[0] == "tail"}
    loops = {}
    for sch in schemes:
        for u in units:
            for direction in ("forward", "inverse"):
                for k in range(3):
                    launch(u, direction, k, sch)
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g):
                    for k in range(20):
                        launch(u, direction, k, sch)
                loops[(sch, u, direction)] = g
    torch.cuda.synchronize()
    per = {key: [] for key in loops}
    for r in range(AB_ROUNDS):
        order = schemes if r % 2 == 0 else schemes[::-1]
        for sch in order:
            for u in units:
                for direction in ("forward", "inverse"):
                    g = loops[(sch, u, direction)]
                    a = torch.cuda.Event(enable_timing=True)
                    b = torch.cuda.Event(enable_timing=True)
                    a.record(stream)
                    g.replay()
                    b.record(stream)
                    torch.cuda.synchronize()
                    per[(sch, u, direction)].append(a.elapsed_time(b) / 20)

    def stats(v):
        v = np.asarray(v)
        return dict(median=round(float(np.median(v)), 5), p10=round(float(np.percentile(v, 10)), 5),
                    p90=round(float(np.percentile(v, 90)), 5))

    out = {"protocol": f"{AB_STEPS} single steps (host calls) per scheme, alternating A/B "
                       f"(order swapped every step), then (FP32 storage) {AB_ROUNDS} alternating "
                       f"rounds of 20-launch loops per chain launch; same buffers, same process"}
    for sch in schemes:
        out[sch] = dict(step_ms=stats(step_ms[sch]),
                        gpixel_s_at_median=round(W * H / (np.median(step_ms[sch]) * 1e-3) / 1e9, 3),
                        launch_ms={f"{u[0]} {u[1]}" + (f"-{u[1] + u[2] - 1}" if u[2] > 1 else "")
                                   + f" {d}": stats(per[(sch, u, d)])
                                   for u in units for d in ("forward", "inverse")})
    diff = step_ms["nonseparable"] - step_ms["separable"]   # paired by step index
    out["step_ms_nonseparable_minus_separable"] = stats(diff)
    del sets, loops
    torch.cuda.empty_cache()
    return out


def load_traffic(kernel_key: str):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except (OSError, ValueError):
        return None
    ent = data.get(kernel_key)
    if not ent or ent.get("kernel_source_sha") != kernel_source_sha():
        return None
    return ent.get("bytes_per_launch")


def copy_reference_gbs(reps=10, pairs=2):
    """Copy bandwidth (read plus write bytes per second) of 1 GiB device
    buffers, alternating over 4 GiB so that they come from HBM; 1 GiB per
    copy, so launch gaps do not count. Two copies are timed, the runtime's
    device-to-device copy and PyTorch's vectorized elementwise kernel (y = x * 1),
    and the faster one is returned with its name: the practical ceiling the
    level kernels are compared with."""
    import torch
    n = 256 << 20
    bufs = [(torch.ones(n, device="cuda"), torch.empty(n, device="cuda")) for _ in range(pairs)]
    ways = {"runtime device copy": lambda a, b: b.copy_(a),
            "elementwise kernel": lambda a, b: torch.mul(a, 1.0, out=b)}
    stream = torch.cuda.current_stream()
    best = (0.0, "")
    for name, fn in ways.items():
        for a, b in bufs:
            fn(a, b)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for k in range(reps):
            a, b = bufs[k % pairs]
            fn(a, b)
        e1.record(stream)
        torch.cuda.synchronize()
        gbs = 2 * 4 * n / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9
        best = max(best, (gbs, name))
    del bufs
    torch.cuda.empty_cache()
    return best


def cpu_baseline(x64, wavelet, levels, seconds):
    import numpy as np
    import oracle
    threads = len(os.sched_getaffinity(0))
    oracle.forward(x64[:64, :64].copy(), wavelet, 1, nthreads=threads)  # load/build
    reps, t0, coef = 0, time.perf_counter(), None
    while True:
        coef = oracle.forward(x64, wavelet, levels, nthreads=threads)
        oracle.inverse(coef, wavelet, levels, nthreads=threads)
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    # the same work on one thread, for at least a third of that time
    reps1, t1 = 0, time.perf_counter()
    while True:
        c1 = oracle.forward(x64, wavelet, levels, nthreads=1)
        oracle.inverse(c1, wavelet, levels, nthreads=1)
        reps1 += 1
        el1 = time.perf_counter() - t1
        if el1 >= seconds / 3:
            break
    H, W = x64.shape
    cpu_model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(value=W * H * reps / el / 1e9, unit="Gpixel/s", cores=threads,
                kind="oracle",
                sample=(f"{reps} x (forward + inverse) of the same {W}x{H} image, "
                        f"{wavelet}, {levels} levels, FP64, OpenMP over rows/columns, "
                        f"{el:.1f} s; host CPU: {cpu_model}"),
                single_thread=dict(value=W * H * reps1 / el1 / 1e9, unit="Gpixel/s", cores=1,
                                   reps=reps1, seconds=round(el1, 2))), coef


def run_batch_workload(args):
    """256 uneven images (sides log-uniform in [64, 4096], multiples of 32),
    3-level forward, planned once: each level is one launch over all images
    per tile configuration in use, captured in one graph. Times the default
    tiles with one workgroup per tile and with a persistent grid, the
    per-class tuned tiles with the faster grid, then levels 1 and 2 fused into
    one head launch over all images (both grids) with the tuned tiles after.
    The spot parity check runs on the last plan's outputs. hbm_frac counts the
    per-level method's bytes throughout."""
    import numpy as np
    import torch
    import synthetic
    from paper_1705_08266_amd import autotune
    from paper_1705_08266_amd.batch import BatchPlan

    L = args.levels
    tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[args.dtype]
    sizes = synthetic.batch_sizes(args.batch, 64, 4096, 32, seed=synthetic.SEED_BASE + 4)
    print(f"[bench] batch of {len(sizes)} images, {sum(w * h for w, h in sizes) / 1e6:.1f} Mpx, "
          f"L={L}", file=sys.stderr, flush=True)
    imgs = []
    for i, (w, h) in enumerate(sizes):
        x = synthetic.uniform_image(h, w, seed=synthetic.SEED_BASE + 4 + i)
        imgs.append(torch.from_numpy(x).to("cuda").to(tdt))
    es = {"f32": 4, "f16": 2, "bf16": 2}[args.dtype]
    alg = sum(sum(level_bytes(w, h, L, es)) for w, h in sizes)

    def time_plan(plan):
        plan.capture()
        for _ in range(args.warmup):
            plan.replay()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            plan.replay()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    runs = {}
    for name, persistent in (("one_workgroup_per_tile", False), ("persistent", True)):
        plan = BatchPlan.forward(imgs, L, args.wavelet, args.scheme, None, persistent)
        ms = time_plan(plan)
        runs[name] = dict(ms=round(ms, 5), gpixel_s=round(plan.pixels / ms / 1e6, 3),
                          hbm_frac=round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          launches_per_level=plan.launches()[1])
        print(f"[bench] default tiles, {name}: {ms:.4f} ms", file=sys.stderr, flush=True)
        del plan
    grid = min(runs, key=lambda k: runs[k]["ms"])
    print("[bench] tuning tiles per size class", file=sys.stderr, flush=True)
    class_tiles = autotune.tune(args.wavelet, args.scheme, args.dtype, L, cache_path=None)
    plan = BatchPlan.forward(imgs, L, args.wavelet, args.scheme, class_tiles,
                             grid == "persistent")
    ms_tuned = time_plan(plan)
    runs["tuned_tiles"] = dict(ms=round(ms_tuned, 5), grid=grid, class_tiles=class_tiles,
                               gpixel_s=round(plan.pixels / ms_tuned / 1e6, 3),
                               launches_per_level=plan.launches()[1])
    if L >= 2:
        # levels 1 and 2 of every image in one head launch, the tuned tiles
        # for the levels after
        for name, persistent in (("head_one_workgroup_per_tile", False), ("head_persistent", True)):
            del plan
            plan = BatchPlan.forward(imgs, L, args.wavelet, args.scheme, class_tiles, persistent,
                                     fuse_head=True)
            ms_h = time_plan(plan)
            runs[name] = dict(ms=round(ms_h, 5), class_tiles=class_tiles,
                              gpixel_s=round(plan.pixels / ms_h / 1e6, 3),
                              hbm_frac=round(alg / (ms_h * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                              launches_per_level=plan.launches()[1])
            print(f"[bench] head + tuned tiles, {name}: {ms_h:.4f} ms", file=sys.stderr,
                  flush=True)
    best = min(runs.values(), key=lambda r: r["ms"])
    ms = best["ms"]
    px = plan.pixels
    # spot parity: the largest image against the oracle
    import oracle
    k = max(range(len(imgs)), key=lambda i: imgs[i].numel())
    ref = oracle.forward(imgs[k].float().cpu().numpy().astype(np.float64), args.wavelet, L,
                         nthreads=len(os.sched_getaffinity(0)))
    err = float(np.abs(plan.outputs[k].float().cpu().numpy() - ref).max() / 255.0)
    print(json.dumps(dict(
        metric=f"Gpixel/s batched {L}-level {args.wavelet} forward, {len(sizes)} uneven images",
        value=round(px / (ms * 1e-3) / 1e9, 3), unit="Gpixel/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(ms, 5), higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype=args.dtype, data="synthetic",
        config=dict(workload=f"{len(sizes)} images, sides log-uniform in [64, 4096] (multiples "
                             f"of 32), uniform integers 0..255, {L} levels forward, planned "
                             f"once, one captured graph", images=len(sizes), pixels=px,
                    levels=L),
        hbm_frac=round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), algorithmic_bytes=alg,
        runs=runs, max_err_rel_largest_image=err)), flush=True)


SERVE_REQUESTS = 5000          # requests per served trace
SERVE_POOL = 256               # distinct resident inputs the requests draw from
SERVE_BUDGET = 64 << 30        # admission budget (bytes)
SERVE_SMALL_BUDGET = 4 << 30   # a budget small enough that admission queues
SERVE_ITERATION_MPX = 1024     # per-iteration cap on level-input pixels (Mpx; 0: none)


def serve_workload_text(n, dtype, cap_mpx=SERVE_ITERATION_MPX, heads=True):
    return (f"{n} requests drawn from {SERVE_POOL} resident inputs, square sides log-uniform "
            f"in [256, 8192] (multiples of 64), levels 1..6, forward/inverse 50/50, {dtype} "
            f"storage with FP32 intermediates, Poisson arrivals, {SERVE_BUDGET >> 30} GiB "
            f"admission budget" + (f", at most {cap_mpx:g} Mpx of level input per iteration"
                                   if cap_mpx else "")
            + (", two levels per step in fused head launches" if heads else
               ", one level per step"))


def run_serve_workload(args):
    """Continuous batching of a Poisson stream of mixed requests (see
    serve_measure): saturation throughput, then p50/p99/p99.9 latency, rate
    and device-busy fraction at 0.5, 0.8 and 0.95 of it, and at 0.8 with a
    4 GiB admission budget."""
    n, px, sat, sweep, small = serve_measure(args, args.requests, args.dtype, (0.5, 0.8, 0.95))
    print(json.dumps(dict(
        metric="Gpixel/s serving throughput, continuous batching of mixed requests",
        value=sat["gpixel_per_s"], unit="Gpixel/s", n_gpus=1, steps=n, warmup=n,
        ms_per_step=None, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype=args.dtype, data="synthetic",
        config=dict(workload=serve_workload_text(n, args.dtype, args.serve_cap,
                                                 args.serve_heads == "on"), requests=n,
                    pixels=px,
                    iteration_cap_mpx=args.serve_cap or None),
        saturation=sat, latency_sweep=sweep, small_budget=small)), flush=True)


def run_ab_workload(args):
    """Two builds of the library in one process: the package's libdwt2.so (A)
    and --other-lib (B), each loaded through its C ABI, alternate in rounds of
    forward+inverse steps on the same buffers (order swapped every round),
    after a check that both give the same bits. For design choices whose
    effect is smaller than the spread between GPUs of the same kind."""
    import ctypes
    import statistics
    import torch
    from paper_1705_08266_amd import _lib

    if not args.other_lib:
        print("--workload ab needs --other-lib PATH (another build of libdwt2.so)", file=sys.stderr)
        sys.exit(2)

    def load(path):
        lib = ctypes.CDLL(path, mode=ctypes.RTLD_LOCAL)
        for f in (lib.dwt2_forward, lib.dwt2_inverse):
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_void_p, ctypes.POINTER(_lib.Desc), ctypes.c_void_p,
                          ctypes.POINTER(_lib.Desc), ctypes.c_int, ctypes.c_int32, ctypes.c_int,
                          ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        lib.dwt2_workspace_bytes.restype = ctypes.c_size_t
        lib.dwt2_workspace_bytes.argtypes = [ctypes.c_int32] * 3 + [ctypes.c_int]
        return lib

    paths = [_lib.LIB_PATH, os.path.abspath(args.other_lib)]
    libs = [load(p) for p in paths]
    W, H = (int(v) for v in args.size.lower().split("x"))
    L = args.levels
    code = {"f32": _lib.F32, "f16": _lib.F16, "bf16": _lib.BF16}[args.dtype]
    tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[args.dtype]
    wav = 0 if args.wavelet == "cdf97" else 1
    sch = 0 if args.scheme == "nonseparable" else 1
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev).manual_seed(0)
    x = (torch.rand(H, W, device=dev, generator=gen) * 255).to(tdt)
    wsb = int(libs[0].dwt2_workspace_bytes(W, H, L, code))
    sets = [(x.clone(), torch.empty_like(x), torch.empty_like(x),
             torch.empty(wsb // 4 + 1, device=dev)) for _ in range(buffer_sets(args, W, H))]
    d = _lib.Desc(W, H, W, code)
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def step(lib, k):
        src, coef, rec, ws = sets[k % len(sets)]
        for st in (lib.dwt2_forward(src.data_ptr(), ctypes.byref(d), coef.data_ptr(),
                                    ctypes.byref(d), wav, L, 0, sch, ws.data_ptr(), wsb, sp),
                   lib.dwt2_inverse(coef.data_ptr(), ctypes.byref(d), rec.data_ptr(),
                                    ctypes.byref(d), wav, L, 0, sch, ws.data_ptr(), wsb, sp)):
            if st != 0:
                raise RuntimeError(f"library call failed with status {st}")

    outs = []
    for lib in libs:
        step(lib, 0)
        torch.cuda.synchronize()
        outs.append((sets[0][1].clone(), sets[0][2].clone()))
    same = bool(torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1]))
    rounds, per = 30, max(1, args.steps // 10)
    us = [[], []]
    for rnd in range(rounds):
        for i in ((0, 1) if rnd % 2 == 0 else (1, 0)):
            for k in range(len(sets)):
                step(libs[i], k)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            a.record()
            for k in range(per):
                step(libs[i], k)
            b.record()
            torch.cuda.synchronize()
            us[i].append(a.elapsed_time(b) / per * 1e3)

    def spread(v):
        v = sorted(v)
        return dict(median=round(statistics.median(v), 3), p10=round(v[len(v) // 10], 3),
                    p90=round(v[9 * len(v) // 10], 3))
    diff = [p - q for p, q in zip(us[0], us[1])]
    med = statistics.median(us[0])
    print(json.dumps(dict(
        metric="us per forward+inverse step, two builds alternating in one process",
        value=round(med, 3), unit="us", n_gpus=1, steps=rounds * per, warmup=len(sets),
        ms_per_step=round(med / 1e3, 5), higher_is_better=False, scaling="weak",
        vs_baseline=None, dtype=args.dtype, data="synthetic",
        config=dict(workload=(f"{W}x{H} uniform image, {args.dtype} storage, {args.wavelet} "
                              f"forward+inverse, {L} levels, {args.scheme} lifting, {rounds} "
                              f"alternating rounds of {per} steps"),
                    a=paths[0], b=paths[1]),
        bit_identical=same, a_us=spread(us[0]), b_us=spread(us[1]),
        a_minus_b_us=spread(diff))), flush=True)


def serve_measure(args, n, dtype, fractions):
    """Serving runs of n requests drawn (seeded) from a pool of SERVE_POOL
    request shapes whose inputs are resident on the device and reused:
    saturation (all offered at time zero), Poisson arrivals at the given
    fractions of the saturation rate, and at 0.8 of it under a budget small
    enough that admission queues. Returns (requests, pixels, saturation,
    {fraction: result}, small-budget result)."""
    import numpy as np
    import torch
    import synthetic
    import paper_1705_08266_amd as dwt
    from paper_1705_08266_amd import serving as sv

    tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[dtype]
    shapes = synthetic.request_stream(SERVE_POOL, 1.0, seed=synthetic.SEED_BASE + 5)
    pool = []
    for t in shapes:
        x = synthetic.device_uniform_image(t.side, t.side, t.seed, tdt)
        pool.append(dwt.forward(x, args.wavelet, t.levels) if t.inverse else x)
    pick = np.random.default_rng(synthetic.SEED_BASE + 7).integers(0, SERVE_POOL, size=n)
    reqs = [sv.Request(i, 0.0, shapes[k].side, shapes[k].side, shapes[k].levels,
                       shapes[k].inverse) for i, k in enumerate(pick)]
    inputs = {i: pool[k] for i, k in enumerate(pick)}
    torch.cuda.synchronize()
    px = sum(r.width * r.height for r in reqs)
    print(f"[bench] serve: {n} requests from {SERVE_POOL} inputs, {px / 1e6:.0f} Mpx, {dtype}",
          file=sys.stderr, flush=True)

    def serve(rate, budget, sub=None):
        rs = reqs if sub is None else reqs[:sub]
        cap = getattr(args, "serve_cap", SERVE_ITERATION_MPX)
        srv = sv.Server(budget_bytes=budget, wavelet=args.wavelet, scheme=args.scheme,
                        dtype=dtype, max_iteration_pixels=int(cap * 1e6) if cap else None,
                        fuse_heads=getattr(args, "serve_heads", "on") == "on")
        if rate is None:
            res = srv.run(rs, inputs, realtime=False)
        else:
            rng = np.random.default_rng(synthetic.SEED_BASE + 6)
            t = np.cumsum(rng.exponential(1.0 / rate, size=len(rs)))
            timed = [sv.Request(r.rid, float(t[i]), r.width, r.height, r.levels, r.inverse)
                     for i, r in enumerate(rs)]
            res = srv.run(timed, inputs, realtime=True)
        torch.cuda.synchronize()
        sm = sv.summarize(res, lambda rid: reqs[rid].width * reqs[rid].height)
        out = dict(requests=len(rs), completed=sm["completed"], rejected=sm["rejected"],
                   requests_per_s=round(sm["requests_per_s"], 1),
                   gpixel_per_s=round(sm["gpixel_per_s"], 3),
                   p50_ms=round(sm["p50_ms"], 3), p99_ms=round(sm["p99_ms"], 3),
                   p999_ms=round(sm["p999_ms"], 3),
                   busy_frac=round(srv.busy_s / sm["span_s"], 4),
                   iterations=srv.iterations, launch_calls=srv.launch_calls,
                   peak_admitted_gib=round(srv.sched.peak_used / 2**30, 2),
                   budget_gib=round(budget / 2**30, 1))
        print(f"[bench] serve rate={rate} budget={budget >> 30} GiB: {out}", file=sys.stderr,
              flush=True)
        return out

    serve(None, SERVE_BUDGET, sub=min(n, 500))       # warm-up: allocator, kernel loads
    sat = serve(None, SERVE_BUDGET)
    sweep = {}
    for f in fractions:
        sweep[str(f)] = dict(offered_per_s=round(f * sat["requests_per_s"], 1),
                             **serve(f * sat["requests_per_s"], SERVE_BUDGET))
    small = dict(offered_per_s=round(0.8 * sat["requests_per_s"], 1),
                 **serve(0.8 * sat["requests_per_s"], SERVE_SMALL_BUDGET))
    del inputs, pool
    torch.cuda.empty_cache()
    return n, px, sat, sweep, small


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--size", default="4096x4096", help="WIDTHxHEIGHT")
    ap.add_argument("--levels", type=int, default=5)
    ap.add_argument("--wavelet", default="cdf97", choices=["cdf97", "cdf53"])
    ap.add_argument("--scheme", default="nonseparable", choices=["nonseparable", "separable"])
    ap.add_argument("--dtype", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--image", default="sinusoid", choices=["sinusoid", "uniform"])
    ap.add_argument("--sets", type=int, default=None,
                    help="rotating buffer sets (default: images of all sets >= 512 MB, "
                         "twice the Infinity Cache; 4..64)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-separable", action="store_true")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving latency measurement of the default workload")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the schemes whose every neighbour exchange goes through LDS")
    ap.add_argument("--graph", action="store_true",
                    help="time replays of one captured graph per step instead of host calls")
    ap.add_argument("--requests", type=int, default=SERVE_REQUESTS,
                    help="requests in the serve workload")
    ap.add_argument("--serve-cap", type=float, default=SERVE_ITERATION_MPX,
                    help="serving: per-iteration cap on level-input pixels, Mpx (0: none)")
    ap.add_argument("--serve-heads", default="on", choices=["on", "off"],
                    help="serving: two levels per step in fused head launches (on) or one")
    ap.add_argument("--fuse", default="auto", choices=["auto", "off"],
                    help="auto: the library fuses the coarse levels; off: one launch per level")
    ap.add_argument("--workload", default="image", choices=["image", "batch", "serve", "ab"],
                    help="image: one image forward+inverse (headline); batch: many uneven "
                         "images, batched forward; serve: continuous batching; ab: this build "
                         "against --other-lib, alternating in one process")
    ap.add_argument("--other-lib", default=None,
                    help="ab workload: path of another build of libdwt2.so")
    ap.add_argument("--batch", type=int, default=256, help="images in the batch workload")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run 4 device copies of 64 MiB (reference kernel of known "
                         "traffic for counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library runs a transform on one device and "
              "does not shard it across GPUs. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        if args.levels == 5 and "--levels" not in sys.argv:
            args.levels = 3
        run_batch_workload(args)
        return
    if args.workload == "ab":
        run_ab_workload(args)
        return
    if args.workload == "serve":
        if "--dtype" not in sys.argv:
            args.dtype = "f16"
        run_serve_workload(args)
        return

    import numpy as np
    import synthetic

    W, H = (int(v) for v in args.size.lower().split("x"))
    L = args.levels
    x = make_image(W, H, args.image, synthetic.SEED_BASE + 2)
    print(f"[bench] {W}x{H} {args.image} {args.dtype} {args.wavelet} L={L} "
          f"{args.scheme}: warmup {args.warmup}, steps {args.steps}", file=sys.stderr,
          flush=True)
    if args.calibrate_copy:
        import torch
        a = torch.empty(16 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(4):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    main_run = run_gpu(args, x, args.scheme)
    sep_run = None
    if not args.no_separable and args.scheme != "separable":
        print("[bench] separable-lifting kernel, same protocol", file=sys.stderr, flush=True)
        sep_run = run_gpu(args, x, "separable")

    ab = None
    if not args.no_separable and args.scheme == "nonseparable":
        print("[bench] interleaved A/B: non-separable vs separable", file=sys.stderr, flush=True)
        ab = ab_schemes(args, x)

    ablation = {}
    if not args.no_ablation and args.dtype == "f32" and args.scheme in ("nonseparable", "separable"):
        # both schemes with every neighbour exchange through LDS and a barrier
        # (the setting of the paper's barrier argument): 2 vs 4 barriers per pair
        for sch in ("nonseparable_lds", "separable_lds"):
            print(f"[bench] exchange ablation: {sch}", file=sys.stderr, flush=True)
            r = run_gpu(args, x, sch)
            ablation[sch] = r

    copy_gbs, copy_kind = copy_reference_gbs()
    es = {"f32": 4, "f16": 2, "bf16": 2}[args.dtype]
    lb = level_bytes(W, H, L, es)
    K = args.steps
    ms_step = main_run["total_ms"] / K
    gpx = W * H / (ms_step * 1e-3) / 1e9
    alg_bytes_step = 2 * sum(lb)

    # the dominant kernel is the chain's first launch: the fused levels 1-2
    # (head), the level-1 launch, or the fused launch of every level (small
    # images); its bytes are that launch's algorithmic bytes
    f1, i1 = main_run["fwd_level_ms"][0], main_run["inv_level_ms"][0]
    dom = "inverse" if i1 > f1 else "forward"
    dom_ms = max(f1, i1)
    unit0 = main_run["units"][0]
    # the head of a 16-bit chain is timed as the two-level call, whose
    # level-2 LL is stored in the storage type
    stand_in = unit0[0] == "head" and args.dtype != "f32"
    dom_bytes = unit_bytes(W, H, 2 if stand_in else L, es, unit0)
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    import paper_1705_08266_amd as dwt
    _, qpl, rows, waves, _, _ = dwt.tile_configs(args.wavelet)[dwt.default_tile(W, H)]
    unit_name = {"head": "fused levels 1-2", "level": "level 1",
                 "tail": f"fused levels 1-{L}"}[unit0[0]]
    kernel_key = (f"{dom}_{unit0[0]}1_{args.wavelet}_{args.scheme}_{args.dtype}_{W}x{H}"
                  + (f"_q{qpl}r{rows}w{waves}" if unit0[0] == "level" else ""))
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=load_traffic(kernel_key),
                    kernel=f"{dom} {unit_name} ({args.scheme})",
                    bytes_per_launch=dom_bytes, avg_launch_ms=round(dom_ms, 5),
                    timed_as=("the two-level call with tiles [HEAD, HEAD] (its level-2 LL in "
                              "the storage type)" if stand_in else "the chain's own launch"),
                    copy_gbs=round(copy_gbs, 1), copy_kind=f"{copy_kind}, 1 GiB",
                    frac_of_copy=round(achieved / copy_gbs, 4))

    def rounded(v):
        return [None if t is None else round(t, 5) for t in v]

    result = dict(
        metric=METRIC, value=round(gpx, 3), unit="Gpixel/s", n_gpus=1, steps=K,
        warmup=args.warmup, ms_per_step=round(ms_step, 5), higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype=args.dtype, data="synthetic",
        config=dict(workload=(f"{W}x{H} {args.image} image, {args.dtype} storage, "
                              f"{args.wavelet} forward+inverse, {L} levels, "
                              f"{args.scheme} lifting, {buffer_sets(args, W, H)} rotating "
                              f"buffer sets"),
                    width=W, height=H, levels=L, wavelet=args.wavelet, scheme=args.scheme,
                    storage=args.dtype, buffer_sets=buffer_sets(args, W, H), fuse=args.fuse),
        roofline=roofline,
        hbm_frac_whole_step=round(alg_bytes_step / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        algorithmic_bytes_per_step=alg_bytes_step,
        executed_bytes_per_step=2 * executed_bytes(W, H, L, es, len(main_run["fused_levels"]),
                                                   main_run["head"]),
        launch_ms=dict(launches=[f"{k} {j}" + (f"-{j + n - 1}" if n > 1 else "")
                                 for k, j, n in main_run["units"]],
                       forward=rounded(main_run["fwd_level_ms"]),
                       inverse=rounded(main_run["inv_level_ms"])),
        fused_levels=dict(head=[1, 2] if main_run["head"] else [],
                          tail=main_run["fused_levels"]),
        launch=("one captured HIP graph per step (forward + inverse chain)"
                if main_run["graph"] else "host calls of the library on one stream"),
        graph_replay=dict(
            per_step=dict(value=round(W * H / (main_run["graph_ms"]["per_step"] * 1e-3) / 1e9, 3),
                          ms_per_step=round(main_run["graph_ms"]["per_step"], 5)),
            multi_step=dict(value=round(W * H / (main_run["graph_ms"]["multi_step"] * 1e-3) / 1e9,
                                        3),
                            ms_per_step=round(main_run["graph_ms"]["multi_step"], 5),
                            steps_per_graph=main_run["graph_ms"]["steps_per_graph"]),
            note="the same steps replayed from captured graphs: one graph per step, or one "
                 "graph holding a step on every buffer set"),
        two_streams=(None if main_run["concurrent_ms"] is None else dict(
            value=round(W * H / (main_run["concurrent_ms"] / K * 1e-3) / 1e9, 3),
            ms_per_step=round(main_run["concurrent_ms"] / K, 5),
            note="the same steps, consecutive ones (independent images) on two streams")),
        graph_replay_matches_eager=main_run["replay_matches_eager"],
    )
    sm = main_run["step_ms"]
    if sm:
        def pct(q):
            return round(sm[min(len(sm) - 1, int(q * len(sm)))], 5)
        result["step_ms"] = dict(median=pct(0.5), p10=pct(0.1), p90=pct(0.9), samples=len(sm),
                                 note="single steps, each between its own events")
    if main_run["warm_ms"]:
        result["warm_cache"] = dict(
            value=round(W * H / (main_run["warm_ms"] * 1e-3) / 1e9, 3),
            ms_per_step=round(main_run["warm_ms"], 5),
            note="one buffer set replayed: the image and coefficients stay in the Infinity Cache")
    if sep_run is not None:
        s_ms = sep_run["total_ms"] / K
        s1 = max(sep_run["fwd_level_ms"][0], sep_run["inv_level_ms"][0])
        result["separable"] = dict(
            value=round(W * H / (s_ms * 1e-3) / 1e9, 3), ms_per_step=round(s_ms, 5),
            first_launch_gbs=round(unit_bytes(W, H, L, es, sep_run["units"][0])
                                   / (s1 * 1e-3) / 1e9, 1),
            launch_ms=dict(forward=rounded(sep_run["fwd_level_ms"]),
                           inverse=rounded(sep_run["inv_level_ms"])))

    if ab is not None:
        result["scheme_ab"] = ab

    if ablation:
        result["exchange_ablation"] = {
            sch: dict(value=round(W * H / (r["total_ms"] / K * 1e-3) / 1e9, 3),
                      ms_per_step=round(r["total_ms"] / K, 5),
                      level1_ms=dict(forward=round(r["fwd_level_ms"][0], 5),
                                     inverse=round(r["inv_level_ms"][0], 5)),
                      barriers_per_lifting_pair=2 if sch.startswith("nonsep") else 4)
            for sch, r in ablation.items()}

    if not args.no_serving and (W, H, L) == (4096, 4096, 5) and args.dtype == "f32":
        # the serving half of the metric: the serving workload (FP16 storage),
        # saturation, then latency at 0.5, 0.8 and 0.95 of it
        n, px, sat, sweep, small = serve_measure(args, SERVE_REQUESTS, "f16", (0.5, 0.8, 0.95))
        at = sweep["0.8"]
        result["serving"] = dict(
            workload=serve_workload_text(n, "f16", heads=args.serve_heads == "on"),
            saturation_gpixel_per_s=sat["gpixel_per_s"],
            saturation_requests_per_s=sat["requests_per_s"],
            offered_per_s=at["offered_per_s"], gpixel_per_s=at["gpixel_per_s"],
            p50_ms=at["p50_ms"], p99_ms=at["p99_ms"], p999_ms=at["p999_ms"],
            busy_frac=at["busy_frac"], requests=n,
            sweep={f: {k: v[k] for k in ("offered_per_s", "requests_per_s", "gpixel_per_s",
                                         "p50_ms", "p99_ms", "p999_ms", "busy_frac")}
                   for f, v in sweep.items()},
            small_budget={k: small[k] for k in ("budget_gib", "offered_per_s", "requests_per_s",
                                                "p50_ms", "p99_ms", "p999_ms",
                                                "peak_admitted_gib")})

    x_stored = main_run["stored"].astype(np.float64)
    scale = float(np.abs(x_stored).max())
    if not args.no_cpu_baseline:
        print(f"[bench] oracle on host cores, ~{args.cpu_seconds:.0f} s", file=sys.stderr,
              flush=True)
        cb, ref = cpu_baseline(x_stored, args.wavelet, L, args.cpu_seconds)
        result["cpu_baseline"] = cb
        result["max_err_rel"] = dict(
            forward=float(np.abs(main_run["coef"] - ref).max() / scale),
            round_trip=float(np.abs(main_run["rec"] - x_stored).max() / scale))
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
