"""Autotuner for the tracer's launch configuration.

The tracer's results never depend on its tuning (rtsdf_trace_tuning), only its
speed does.  `tune` times candidate settings on the caller's own pipeline (or
batch) with HIP events, keeps the fastest, applies it with
``rtsdf_trace_config`` and remembers it in a JSON cache keyed by GPU
architecture, fine-grid size, triangle-count bucket and rays per texel.  The
accumulation state touched while timing is reset afterwards.
"""
from __future__ import annotations

import itertools
import json
import math
import os

import torch

from . import rtsdf as R

DEFAULT_CACHE = os.environ.get("RTSDF_AUTOTUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "rtsdf_autotune.json"))

SPACE = {
    "refill": (8, 16),
    "stack_lds": (12, 16, 24),
    "bin_directions": (0, 1),
    "loop": (2, 3),
    "blocks_per_cu": (0,),
}


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName
    except Exception:
        return "unknown"


def cache_key(nf: int, triangles: int, rays: int) -> str:
    bucket = int(math.log2(max(triangles, 1)))
    return f"{_arch()}|nf{nf}|tri2^{bucket}|r{rays}"


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(entries: dict, path: str = DEFAULT_CACHE):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(entries, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def candidates(space: dict = SPACE):
    keys = list(space)
    for vals in itertools.product(*(space[k] for k in keys)):
        yield dict(zip(keys, vals))


def _time(fn, reps: int) -> float:
    stream = torch.cuda.current_stream()
    fn()  # warm-up
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        fn()
    stop.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / reps


def tune(target, reps: int = 2, space: dict = SPACE, cache: str | None = DEFAULT_CACHE, force: bool = False) -> dict:
    """Pick the fastest tracer tuning for `target` (a Pipeline or a rtsdf.Batch).

    Returns {"tuning": {...}, "ms": best time, "trials": [(tuning, ms), ...]}.
    """
    from .pipeline import Pipeline

    if isinstance(target, Pipeline):
        key = cache_key(target.nf, int(target.faces.shape[0]), target.rays)
        target.step(0)  # coarse stages and selection once; timing repeats the trace only
        frame = [1]

        def run():
            target.trace(frame[0])
            frame[0] += 1

        def reset():
            target.reset()
    else:
        key = f"{_arch()}|batch{target.n}"
        frame = [0]

        def run():
            target.step(frame[0])
            frame[0] += 1

        def reset():
            target.reset()

    entries = load_cache(cache) if cache else {}
    if not force and key in entries:
        best = entries[key]["tuning"]
        R.rtsdf_trace_config(**best, stats=0)
        return {"tuning": best, "ms": entries[key]["ms"], "trials": [], "cached": True}
    trials = []
    for cand in candidates(space):
        R.rtsdf_trace_config(**cand, stats=0)
        trials.append((cand, _time(run, reps)))
    best, ms = min(trials, key=lambda t: t[1])
    R.rtsdf_trace_config(**best, stats=0)
    reset()
    torch.cuda.synchronize()
    if cache:
        entries[key] = {"tuning": best, "ms": ms}
        save_cache(entries, cache)
    return {"tuning": best, "ms": ms, "trials": trials, "cached": False}
