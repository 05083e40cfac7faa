"""Autotuner for the tracer's launch configuration.

The tracer's results never depend on its tuning (rtsdf_trace_tuning), only its
speed does.  `tune` times candidate settings on the caller's own pipeline (or
batch) with HIP events and keeps the fastest.  The knobs:

* ``blocks_per_cu``  persistent workgroups of four wavefronts per compute unit,
  i.e. traversal wavefronts per SIMD (0 = as many as fit, 6 with the default
  LDS stack);
* ``tile_texels``    texels per wavefront tile (a compact Morton block of the
  fine grid; at most 768 rays);
* ``refill``         free lanes at which a wavefront takes new rays;
* ``stack_lds``      traversal stack entries per lane kept in LDS;
* ``bin_directions`` sorting a tile's rays by direction;
* ``loop``           traversal loop shape (queued triangle tests or the one-fetch loop);
* ``bvh_width``      the two-child hierarchy or its 4-wide copy (single-level
  scenes that refit or stay static; batches and device-rebuilt or two-level
  scenes trace two-wide and skip this knob).

For a Pipeline the jump flooding's two knobs (``rtsdf_jfa_config``: the
near-pass staging, seeds alone or seed pairs in LDS; the far-pass brick order,
slab order, coset order, or coset order in brick pairs or 2 x 2 quads) are
timed too, all eight combinations, and the fastest is kept for the pipeline's
coarse grid size.

The search is coordinate descent from the target's current tuning: each knob
in turn takes each of its values with the others fixed, a change is kept when
it is at least 0.5 % faster, and sweeps repeat until one changes nothing (or
the product of a small space is timed exhaustively).  The winner is applied
to the target only -- the scene of a Pipeline (``rtsdf_scene_set_tuning``) or
the Batch (``rtsdf_batch_set_tuning``) -- never to the process default, and is
remembered in a JSON cache keyed by GPU architecture and workload shape (fine
size, triangle-count bucket and rays per texel; for batches the scene count,
total fine texels, total triangles and the set of ray counts).  The
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

# first value of each knob = the library default
SPACE = {
    "blocks_per_cu": (0, 3, 4, 5),
    "tile_texels": (64, 32, 16),
    "refill": (28, 16),
    "stack_lds": (12, 16, 24),
    "bin_directions": (1, 0),
    "loop": (4, 3),
    "bvh_width": (2, 4),
}


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName
    except Exception:
        return "unknown"


def _bucket(x: int) -> int:
    return int(math.log2(max(int(x), 1)))


def cache_key(nf: int, triangles: int, rays: int) -> str:
    return f"{_arch()}|nf{nf}|tri2^{_bucket(triangles)}|r{rays}"


def batch_cache_key(batch) -> str:
    d = batch.descriptors
    texels = sum(s["fine_n"] ** 3 for s in d)
    tris = sum(s["nt"] for s in d)
    rays = sorted({s["rays"] for s in d})
    return f"{_arch()}|batch{batch.n}|tex2^{_bucket(texels)}|tri2^{_bucket(tris)}|r{','.join(map(str, rays))}"


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


def search(measure, start: dict, space: dict = SPACE, sweeps: int = 3, exhaustive: bool | None = None,
           min_gain: float = 0.005):
    """Minimise measure(tuning) over `space`; returns (best, ms, trials).

    Coordinate descent from `start` (which must hold a value for every knob of the space); with
    `exhaustive` (default: when the space has at most 16 points) every point of the product is timed."""
    if exhaustive is None:
        exhaustive = math.prod(len(v) for v in space.values()) <= 16
    trials = []
    if exhaustive:
        for cand in candidates(space):
            trials.append((cand, measure(cand)))
        best, ms = min(trials, key=lambda t: t[1])
        return best, ms, trials
    best = {k: start[k] for k in space}
    ms = measure(best)
    trials.append((dict(best), ms))
    seen = {tuple(sorted(best.items()))}
    for _ in range(sweeps):
        changed = False
        for knob, values in space.items():
            for v in values:
                cand = {**best, knob: v}
                key = tuple(sorted(cand.items()))
                if key in seen:
                    continue
                seen.add(key)
                t = measure(cand)
                trials.append((cand, t))
                if t < ms * (1.0 - min_gain):
                    best, ms, changed = cand, t, True
        if not changed:
            break
    return best, ms, trials


def tune(target, reps: int = 2, space: dict = SPACE, cache: str | None = DEFAULT_CACHE, force: bool = False,
         sweeps: int = 3, exhaustive: bool | None = None) -> dict:
    """Pick the fastest tracer tuning for `target` (a Pipeline or a rtsdf.Batch) and apply it to that target.

    Returns {"tuning": {...}, "ms": best time, "trials": [(tuning, ms), ...], "cached": bool, "key": str}.
    """
    from .pipeline import Pipeline

    if isinstance(target, Pipeline):
        if target.parts or target.rebuild:  # two-level and device-rebuilt scenes trace two-wide
            space = {k: v for k, v in space.items() if k != "bvh_width"}
        key = cache_key(target.nf, int(target.faces.shape[0]), target.rays)
        current = target.scene.tuning().as_dict()
        target.step(0)  # coarse stages and selection once; timing repeats the trace only
        frame = [1]

        def run():
            target.trace(frame[0])
            frame[0] += 1

        def apply(t):
            target.scene.set_tuning(**t, stats=0)
    else:
        space = {k: v for k, v in space.items() if k != "bvh_width"}  # batches trace two-wide
        key = batch_cache_key(target)
        current = {**R.rtsdf_trace_config_get().as_dict(), **getattr(target, "_tuning", {})}
        frame = [0]

        def run():
            target.step(frame[0])
            frame[0] += 1

        def apply(t):
            target.set_tuning(**t, stats=0)

    entries = load_cache(cache) if cache else {}
    if not force and key in entries:
        best = entries[key]["tuning"]
        apply(best)
        if "jfa_near_stage" in entries[key]:
            R.rtsdf_jfa_config(target.nc, entries[key]["jfa_near_stage"], entries[key].get("jfa_far_order", 0))
        return {"tuning": best, "ms": entries[key]["ms"], "trials": [], "cached": True, "key": key,
                "jfa": entries[key].get("jfa")}

    def measure(t):
        apply(t)
        return _time(run, reps)

    start = {k: current.get(k, v[0]) for k, v in space.items()}
    best, ms, trials = search(measure, start, space, sweeps=sweeps, exhaustive=exhaustive)
    apply(best)
    jfa = tune_jfa(target, reps=max(reps, 3)) if isinstance(target, Pipeline) else None
    target.reset()
    torch.cuda.synchronize()
    if cache:
        entries[key] = {"tuning": best, "ms": ms}
        if jfa is not None:
            entries[key].update(jfa_near_stage=jfa["near_stage"], jfa_far_order=jfa["far_order"], jfa=jfa)
        save_cache(entries, cache)
    return {"tuning": best, "ms": ms, "trials": trials, "cached": False, "key": key, "jfa": jfa}


def tune_jfa(p, reps: int = 3) -> dict:
    """Time the jump flooding of pipeline `p` with each near-pass staging (seeds alone or seed pairs) and each
    far-pass brick order (slab order, coset order, coset order in brick pairs or quads) -- rtsdf_jfa_config; the
    results are the same -- and keep the fastest combination for grids of p's coarse size (process-wide setting).
    Each timed run voxelizes first, the same work for every combination."""
    n = p.nc
    times = {}
    for stage, order in itertools.product((1, 2), (1, 2, 3, 4)):
        R.rtsdf_jfa_config(n, stage, order)

        def run():
            p.voxelize()
            p.jfa()
        times[(stage, order)] = _time(run, reps)
    stage, order = min(times, key=times.get)
    R.rtsdf_jfa_config(n, stage, order)
    return {"near_stage": stage, "far_order": order, "ms": {f"{a},{b}": t for (a, b), t in times.items()}}
