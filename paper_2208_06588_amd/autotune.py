"""Launch-configuration tuner for the batched forward run.

Times short runs of every candidate (engine and stages per launch,
work-group size, graph use, cells per thread, tile form) on copies of the caller's
batch, times the near-fastest again over longer runs and keeps the fastest
(the library's automatic shape when it is within 1 % of it).
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

# Stages per launch: the stage engine runs one RK stage per kernel launch (the
# global LF speed of a stage is a reduction over the whole instance, taken
# between launches); the persistent engine runs 3 x steps_per_launch stages of
# each instance per launch (0: every stage to the end of the run), a
# work-group per instance.
CANDIDATES = [
    dict(engine=alew.ENGINE_PERSISTENT, block=128, steps_per_launch=0, use_graph=0,
         cells_per_thread=1),
    dict(engine=alew.ENGINE_PERSISTENT, block=256, steps_per_launch=0, use_graph=0,
         cells_per_thread=1),
    dict(engine=alew.ENGINE_PERSISTENT, block=64, steps_per_launch=0, use_graph=0,
         cells_per_thread=2),
    dict(engine=alew.ENGINE_PERSISTENT, block=64, steps_per_launch=1, use_graph=0,
         cells_per_thread=2),
    dict(engine=alew.ENGINE_PERSISTENT, block=256, steps_per_launch=1, use_graph=0,
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


# the shape the library picks by itself for the stage engine (block 0 and
# cells_per_thread 0 resolve to one-wave tiles, two cells per thread)
AUTO = dict(engine=alew.ENGINE_STAGES, block=64, steps_per_launch=0, use_graph=1,
            cells_per_thread=2)


def name_of(c) -> str:
    return (f"engine{c['engine']}-b{c['block']}-g{c['use_graph']}"
            f"-c{c.get('cells_per_thread', 1)}-t{c.get('compact_tiles', 0)}"
            f"-s{c.get('steps_per_launch', 0)}")

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

    def time_one(cand, ns):
        ctx.set_launch(**cand)
        # one untimed step builds tile tables and graphs, then `ns` steps timed
        # on the wall clock (launches, host checks between launches and the
        # call's set-up alike for every candidate)
        wall = 0.0
        for nrun in (1, ns):
            T = {k: v.clone() for k, v in state.items()}
            torch.cuda.synchronize()
            a = time.perf_counter()
            ctx.run(p, cell_off, T["h"], T["hu"], T["b"], T["x"], T["xi"], max_steps=[nrun] * ninst)
            torch.cuda.synchronize()
            wall = time.perf_counter() - a
            del T
        return wall

    times = {}
    for cand in candidates:
        name = name_of(cand)
        times[name] = time_one(cand, steps)
        if log:
            log(f"tune {name}: {times[name] * 1e3:.1f} ms for {steps} steps")
    # second round: the candidates within 10 % of the fastest, timed again over
    # twice the steps (best of two), so that near ties are not settled by noise
    t0 = min(times.values())
    final = {}
    for cand in candidates:
        name = name_of(cand)
        if times[name] <= 1.10 * t0:
            final[name] = min(time_one(cand, 2 * steps) for _ in range(2)) / 2
            if log:
                log(f"tune {name}: {final[name] * 1e3:.2f} ms per {steps} steps (second round)")
    best_name = min(final, key=final.get)
    # within 1 % of the fastest, the library's automatic shape is kept
    auto = name_of(AUTO)
    if auto in final and final[auto] <= 1.01 * final[best_name]:
        best_name = auto
    best = next(c for c in candidates if name_of(c) == best_name)
    ctx.set_launch(**best)
    cache[key] = dict(best=best, times=times)
    _store(cache)
    return best, times
