"""Autotuner for batched launches.

Two knobs shape a pool's launches without changing any result:

* islands per workgroup: a step workgroup stages a tile of
  block_threads * agents_per_thread / N whole islands, so the tile is set
  by the workgroup size (64, 128 or 256 threads);
* generations per launch: how many generations one advance enqueues (one
  site-schedule launch plus one step launch per generation, replayed as a
  captured hipGraph or launched directly).

Because results do not depend on either knob, tuning runs online: each
candidate shape advances the real runs once, the wall time per generation
is compared, and the pool keeps the fastest.  No work is thrown away.  The
choice is cached in a JSON file keyed by the run set (path from the
HSGA_AUTOTUNE_CACHE environment variable, default
~/.cache/hsga_autotune.json).
"""
from __future__ import annotations

import hashlib
import json
import os
import time

DEFAULT_CANDIDATES = (
    # (block_threads, generations per launch, hipGraph replay)
    (64, 64, False), (64, 64, True), (128, 64, True), (256, 64, True),
    (64, 256, True), (256, 256, True), (64, 16, True),
)


def cache_path() -> str:
    return os.environ.get("HSGA_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "hsga_autotune.json"))


def signature(specs) -> str:
    """Key of a run set: the sorted launch-relevant parameters of its runs."""
    items = sorted((s.grid_w, s.grid_h, s.pop_per_island, s.surface_sites, s.surface_kind,
                    s.tournament_size, s.migrants_per_island) for s in specs)
    return hashlib.sha256(json.dumps(items).encode()).hexdigest()[:20]


def load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def store_cache(key: str, choice: dict):
    data = load_cache()
    data[key] = choice
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1)
    os.replace(tmp, path)


def tune_online(pool, key: str | None = None, candidates=DEFAULT_CANDIDATES,
                use_cache: bool = True, repeats: int = 2) -> dict:
    """Pick the pool's launch shape while advancing its runs.

    Returns {"block_threads", "gens_per_launch", "use_graph", "trials"}; the
    pool is left set to the choice.  Candidates are tried until the runs
    finish; each is timed over `repeats` advances and its fastest counts; a
    hipGraph candidate's timed advances follow the one that captures the
    graph.  A candidate timed fewer times (the runs ran out) still counts.
    """
    if use_cache and key is not None:
        hit = load_cache().get(key)
        if hit:
            pool.set_launch(hit["block_threads"], hit["use_graph"])
            hit = dict(hit)
            hit["cached"] = True
            return hit
    trials = []
    done = False
    for block, gens, graph in candidates:
        pool.set_launch(block, graph)
        pool.sync()
        if graph:
            if pool.advance(gens) == 0:
                break
            pool.sync()
        # at least two timed advances per candidate (the faster one counts),
        # so that one noisy advance does not decide
        times = []
        for _ in range(repeats):
            t0 = time.perf_counter()
            n = pool.advance(gens)
            pool.sync()
            dt = time.perf_counter() - t0
            if n == 0:
                done = True
                break
            times.append(dt / n)
        if times:
            trials.append({"block_threads": block, "gens_per_launch": gens, "use_graph": graph,
                           "s_per_generation": min(times), "timings": times})
        if done:
            break
    if not trials:
        choice = {"block_threads": 64, "gens_per_launch": 64, "use_graph": False}
    else:
        best = min(trials, key=lambda t: t["s_per_generation"])
        choice = {k: best[k] for k in ("block_threads", "gens_per_launch", "use_graph")}
    pool.set_launch(choice["block_threads"], choice["use_graph"])
    if key is not None and trials:
        store_cache(key, choice)
    choice["trials"] = trials
    choice["cached"] = False
    return choice
