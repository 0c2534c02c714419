"""Per-size-class choice of the tile configuration for planned batches.

Each size class is tuned on its own: a batch of images whose level input
lies in that class, transformed by one level, so that only that class's
configuration is exercised. Every compiled configuration is timed on it
(graph-captured replays, so host overhead does not count) and the fastest
kept. Results are cached in a JSON file keyed by device, wavelet, scheme,
storage type and level count; the level count only keys the cache (a class's
launches look alike at every level).
"""
from __future__ import annotations

import json
import os

from . import tile_configs

# Representative level-input sides of the four size classes (<= 128^2,
# <= 512^2, <= 2048^2, larger).
CLASS_SIDES = (96, 384, 1536, 4096)


def _time_plan(plan, reps=5):
    import torch
    plan.capture()
    for _ in range(2):
        plan.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plan.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def gpu_class_timer(wavelet, scheme, dtype, images_per_class=8):
    """timer(cls, tile) -> ms of a one-level batch of class `cls` images on
    the current GPU with `tile` for that class."""
    import torch
    from .batch import BatchPlan
    tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[dtype]
    gen = torch.Generator(device="cuda").manual_seed(12345)
    cache = {}

    def timer(cls, tile):
        if cls not in cache:
            side = CLASS_SIDES[cls]
            n = images_per_class if side <= 1536 else 2
            cache.clear()   # keep one class's images alive at a time
            cache[cls] = [torch.rand(side, side, device="cuda", generator=gen).mul_(255).to(tdt)
                          for _ in range(n)]
        class_tiles = [0] * len(CLASS_SIDES)
        class_tiles[cls] = tile
        plan = BatchPlan.forward(cache[cls], 1, wavelet, scheme, class_tiles)
        return _time_plan(plan)
    return timer


def tune(wavelet="cdf97", scheme="nonseparable", dtype="f32", levels=1, cache_path=None,
         force=False, verbose=False, timer=None, candidates=None, device_name=None):
    """Return the fastest tile id for each size class.

    cache_path: a JSON file read before and written after tuning (None: no
    cache). force: re-tune even when the cache holds the key. timer,
    candidates, device_name: the per-(class, tile) timer, the tile ids to try
    and the device name of the cache key; by default the current GPU, every
    compiled configuration and that GPU's name."""
    if device_name is None:
        import torch
        device_name = torch.cuda.get_device_name()
    key = f"{device_name}|{wavelet}|{scheme}|{dtype}|L{levels}"
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if not force and key in cache:
        return list(cache[key]["class_tiles"])
    if candidates is None:
        candidates = [c[0] for c in tile_configs(wavelet)]
    if timer is None:
        timer = gpu_class_timer(wavelet, scheme, dtype)
    best, timings = [], {}
    for cls in range(len(CLASS_SIDES)):
        res = {t: float(timer(cls, t)) for t in candidates}
        pick = min(res, key=res.get)
        best.append(pick)
        timings[str(cls)] = {str(t): round(v, 5) for t, v in res.items()}
        if verbose:
            print(f"class {cls} (side {CLASS_SIDES[cls]}): " +
                  ", ".join(f"tile {t} {v * 1000:.1f} us" for t, v in res.items()) +
                  f" -> {pick}", flush=True)
    cache[key] = {"class_tiles": best, "ms": timings}
    if cache_path:
        d = os.path.dirname(cache_path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, cache_path)
    return best


__all__ = ["tune", "CLASS_SIDES", "gpu_class_timer"]
