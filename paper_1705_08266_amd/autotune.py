"""Per-size-class choice of the 2-D tile configuration for batched launches.

For each size class the tuner times every compiled 2-D tile configuration on
a batch of images of that class (graph-captured, so host overhead does not
count) and keeps the fastest. Results are cached in a JSON file keyed by
device, wavelet, scheme, storage type and level count.
"""
from __future__ import annotations

import json
import os

from . import _lib, load, tile_configs
from .batch import BatchPlan

# Representative level-input sides of the four size classes.
CLASS_SIDES = (96, 384, 1536, 4096)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "dwt2_autotune.json")


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


def tune(wavelet="cdf97", scheme="nonseparable", dtype="f32", levels=1, images_per_class=8,
         cache_path=DEFAULT_CACHE, force=False, verbose=False):
    """Return the fastest 2-D tile id for each size class (cached)."""
    import torch
    dev = torch.cuda.get_device_name()
    key = f"{dev}|{wavelet}|{scheme}|{dtype}|L{levels}"
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
    if not force and key in cache:
        return list(cache[key]["class_tiles"])
    tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[dtype]
    cands = [c[0] for c in tile_configs(wavelet)]
    best, timings = [], {}
    gen = torch.Generator(device="cuda").manual_seed(12345)
    for c, side in enumerate(CLASS_SIDES):
        side -= side % (1 << levels)
        n = images_per_class if side <= 1536 else 2
        imgs = [torch.rand(side, side, device="cuda", generator=gen).mul_(255).to(tdt)
                for _ in range(n)]
        res = {}
        for t in cands:
            class_tiles = [t] * _lib.SIZE_CLASSES
            plan = BatchPlan.forward(imgs, levels, wavelet, scheme, class_tiles)
            res[t] = _time_plan(plan)
            del plan
        pick = min(res, key=res.get)
        best.append(pick)
        timings[str(c)] = {str(t): round(v, 5) for t, v in res.items()}
        if verbose:
            print(f"class {c} (side {side}): " +
                  ", ".join(f"tile {t} {v * 1000:.1f} us" for t, v in res.items()) +
                  f" -> {pick}", flush=True)
        del imgs
    cache[key] = {"class_tiles": best, "ms": timings}
    if cache_path:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        json.dump(cache, open(tmp, "w"), indent=1)
        os.replace(tmp, cache_path)
    return best


__all__ = ["tune", "CLASS_SIDES", "load"]
