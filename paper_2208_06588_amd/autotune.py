"""Launch-configuration tuner for the batched forward run.

Times short runs of every candidate (engine, work-group size, graph use /
steps per launch) on copies of the caller's batch and keeps the fastest.
Results are cached in a JSON file keyed by the GPU architecture and a hash of
the batch shape and scheme parameters.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import torch

from . import alew

CANDIDATES = [
    dict(engine=alew.ENGINE_PERSISTENT, block=128, steps_per_launch=0, use_graph=0,
         cells_per_thread=1),
    dict(engine=alew.ENGINE_PERSISTENT, block=256, steps_per_launch=0, use_graph=0,
         cells_per_thread=1),
    dict(engine=alew.ENGINE_STAGES, block=128, steps_per_launch=0, use_graph=1, cells_per_thread=1),
    dict(engine=alew.ENGINE_STAGES, block=256, steps_per_launch=0, use_graph=1, cells_per_thread=1),
    dict(engine=alew.ENGINE_STAGES, block=512, steps_per_launch=0, use_graph=1, cells_per_thread=1),
    dict(engine=alew.ENGINE_STAGES, block=128, steps_per_launch=0, use_graph=1, cells_per_thread=2),
    dict(engine=alew.ENGINE_STAGES, block=256, steps_per_launch=0, use_graph=1, cells_per_thread=2),
    dict(engine=alew.ENGINE_STAGES, block=256, steps_per_launch=0, use_graph=1, cells_per_thread=1,
         compact_tiles=1),
    dict(engine=alew.ENGINE_STAGES, block=64, steps_per_launch=0, use_graph=1, cells_per_thread=1),
    dict(engine=alew.ENGINE_STAGES, block=64, steps_per_launch=0, use_graph=1, cells_per_thread=2),
    dict(engine=alew.ENGINE_STAGES, block=64, steps_per_launch=0, use_graph=1, cells_per_thread=2,
         compact_tiles=1),
]


def name_of(c) -> str:
    return (f"engine{c['engine']}-b{c['block']}-g{c['use_graph']}"
            f"-c{c.get('cells_per_thread', 1)}-t{c.get('compact_tiles', 0)}")

CACHE = os.environ.get("ALEW_TUNE_CACHE", os.path.expanduser("~/.cache/alew/autotune.json"))


def _key(p: alew.Params, cell_off, steps):
    h = hashlib.sha1()
    h.update(bytes(p))
    h.update(str(list(map(int, cell_off))).encode())
    h.update(str(steps).encode())
    arch = torch.cuda.get_device_properties(0).gcnArchName if torch.cuda.is_available() else "cpu"
    return f"{arch}:{h.hexdigest()}"


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        with open(CACHE, "w") as f:
            json.dump(d, f, indent=1)
    except OSError:
        pass


def tune(ctx: alew.Context, p: alew.Params, cell_off, state: dict, steps: int = 2,
         candidates=CANDIDATES, use_cache: bool = True, log=None):
    """Pick the fastest launch configuration for this batch; returns
    (best_config, {config_name: seconds}).  state holds the device tensors
    h, hu, b, x, xi (left untouched)."""
    key = _key(p, cell_off, steps)
    cache = _load() if use_cache else {}
    if key in cache:
        best = cache[key]["best"]
        ctx.set_launch(**best)
        return best, cache[key]["times"]
    ninst = len(cell_off) - 1
    times = {}
    for cand in candidates:
        ctx.set_launch(**cand)
        # one untimed step builds tile tables and graphs, then `steps` timed steps
        for nrun, ns in ((0, 1), (1, steps)):
            T = {k: v.clone() for k, v in state.items()}
            torch.cuda.synchronize()
            ctx.run(p, cell_off, T["h"], T["hu"], T["b"], T["x"], T["xi"], max_steps=[ns] * ninst)
            torch.cuda.synchronize()
            del T
        dt = ctx.last_timing()[0] * 1e-3
        name = name_of(cand)
        times[name] = dt
        if log:
            log(f"tune {name}: {dt * 1e3:.1f} ms for {steps} steps")
    best_name = min(times, key=times.get)
    best = next(c for c in candidates if name_of(c) == best_name)
    ctx.set_launch(**best)
    cache[key] = dict(best=best, times=times)
    _store(cache)
    return best, times
