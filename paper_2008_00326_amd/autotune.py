"""Launch autotuner for the batched scoring path.

The scoring launch has a few free choices that never change a result, only
how the poses are spread over the persistent kernels: the work-group size of
the smallest LDS footprint class (256 or 512 threads), the LDS threshold
that sends a pose to that class, the number of persistent work-groups per
class, whether each class scores its costliest poses first, and whether J_o
regions too large for LDS are keyed in device memory or in LDS row bands.
The tuner times a small candidate set on a sample of the caller's work and
keeps the fastest when it beats the default by at least 5 %, otherwise the
default; the choice is cached as JSON keyed by the device architecture and a
shape bucket (image size, mean mesh size, poses per item, colour term).
"""
from __future__ import annotations

import json
import math
import os
import time

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "perch", "autotune.json")


def device_arch(device: int = 0) -> str:
    import torch
    name = getattr(torch.cuda.get_device_properties(device), "gcnArchName", "") or "unknown"
    return name.split(":")[0]


def shape_bucket(pixels: float, mean_tris: float, mean_poses: float, rgb: bool) -> str:
    """Key of a workload shape: powers of two of the image size, the mean
    triangle count and the mean poses per item, and the colour term."""
    def lg(x):
        return int(round(math.log2(max(x, 1.0))))
    return f"px{lg(pixels)}-tri{lg(mean_tris)}-pose{lg(mean_poses)}-{'rgb' if rgb else 'depth'}"


def candidates(defaults: dict, n_cu: int):
    """The candidate tunings around the context's defaults."""
    out = []
    fit512 = defaults["small_words"] if defaults["small_block"] == 512 else None
    for block in (512, 256):
        for order in (2, 1):
            for frac in (1.0, 0.5):
                c = {"small_block": block, "order": order, "grid": [0, 0, 0, 0], "small_words": 0}
                if frac < 1.0:
                    if block != 512 or fit512 is None:
                        continue
                    c["small_words"] = int(fit512 * frac)
                out.append(c)
    # fewer concurrent device-key work-groups (less L2 pressure)
    out.append({"small_block": 512, "order": 2, "grid": [0, 0, max(n_cu // 2, 1), 0], "small_words": 0})
    # large J_o regions keyed in device memory instead of LDS bands
    out.append({"small_block": 512, "order": 2, "grid": [0, 0, 0, 0], "small_words": 0, "key_bands": 1})
    return out


# A candidate replaces the default only when it is this much faster: the
# choices move a launch by a few per cent at most, which is within the
# box-to-box and run-to-run spread of the timing.
MIN_GAIN = 0.05


def choose(trials, min_gain: float = MIN_GAIN) -> dict:
    """The trial to keep: the fastest if it beats the default (trials[0]) by
    at least `min_gain` of the default's time, otherwise the default."""
    best = min(trials, key=lambda t: t["ms"])
    if best["ms"] <= trials[0]["ms"] * (1.0 - min_gain):
        return best
    return trials[0]


def _time(ctx, items, reps, stream):
    import torch
    ctx.score_batch(items, stream=stream)            # warm-up (also sizes the buffers)
    stream.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    ms = []
    for _ in range(reps):
        a.record(stream)
        ctx.score_batch(items, stream=stream)
        b.record(stream)
        b.synchronize()
        ms.append(a.elapsed_time(b))
    ms.sort()
    return ms[len(ms) // 2]


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: str = DEFAULT_CACHE) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(ctx, items, bucket: str, *, cache_path: str | None = DEFAULT_CACHE, reps: int = 3, stream=None,
             force: bool = False) -> dict:
    """Pick and apply the fastest tuning for `items` (score_batch items).

    Returns {"key", "tuning", "ms", "trials", "cached"}; the chosen tuning is
    left set on the context.  With a cache hit nothing is timed."""
    import torch
    key = f"{device_arch()}|{bucket}"
    cache = load_cache(cache_path) if cache_path else {}
    if not force and key in cache:
        ctx.set_tuning(cache[key]["tuning"])
        return dict(cache[key], key=key, cached=True)
    stream = stream or torch.cuda.current_stream()
    ctx.set_tuning(None)
    defaults = ctx.tuning()
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    trials = []
    t0 = time.perf_counter()
    for c in candidates(defaults, n_cu):
        ctx.set_tuning(c)
        trials.append({"tuning": c, "ms": round(_time(ctx, items, reps, stream), 4)})
    best = choose(trials)
    ctx.set_tuning(best["tuning"])
    fastest = min(trials, key=lambda t: t["ms"])
    rec = {"tuning": best["tuning"], "ms": best["ms"], "trials": trials,
           "default_ms": trials[0]["ms"], "fastest_ms": fastest["ms"],
           "gain_of_fastest": round(1.0 - fastest["ms"] / trials[0]["ms"], 4),
           "seconds": round(time.perf_counter() - t0, 2)}
    if cache_path:
        cache[key] = rec
        save_cache(cache, cache_path)
    return dict(rec, key=key, cached=False)
