"""Autotuner for the batched predation launch.

The persistent launch has two shape parameters: threads per model workgroup
(waves per block) and slots per thread per chunk.  Their best values depend
on the model sizes in the batch (a small model wastes a wide workgroup; a large
one needs many slots in flight).  The tuner times every candidate on a fresh
sample of the actual batch and caches the winner in a JSON file keyed by the
GPU architecture and a caller-chosen workload key.
"""
from __future__ import annotations

import json
import os

import torch

CANDIDATES = ((256, 1), (256, 2), (256, 4), (512, 1), (512, 2), (512, 4), (1024, 2), (1024, 4))


def default_cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "abm_mi355x", "tune.json")


def _arch() -> str:
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(props, "gcnArchName", props.name)


def autotune_batched(make_batch, key: str, steps: int = 8, candidates=CANDIDATES,
                     cache_path: str | None = None, use_cache: bool = True) -> dict:
    """make_batch(block_threads, items) -> a freshly initialised BatchedPredation.
    Returns {"block_threads", "items", "timings_ms": {...}, "cached": bool}."""
    path = cache_path or default_cache_path()
    full_key = f"{_arch()}|{key}"
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
        if full_key in cache:
            hit = dict(cache[full_key])
            hit["cached"] = True
            return hit
    timings = {}
    for block, items in candidates:
        b = make_batch(block, items)
        b.run(1, block_threads=block, items=items)       # warm-up
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.run(steps, block_threads=block, items=items)
        e1.record()
        torch.cuda.synchronize()
        timings[f"{block}x{items}"] = e0.elapsed_time(e1)
        del b
    best = min(timings, key=timings.get)
    block, items = (int(v) for v in best.split("x"))
    result = {"block_threads": block, "items": items, "timings_ms": timings}
    if use_cache:
        cache[full_key] = result
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path + ".tmp", "w") as f:
                json.dump(cache, f, indent=1)
            os.replace(path + ".tmp", path)
        except OSError:
            pass
    out = dict(result)
    out["cached"] = False
    return out
