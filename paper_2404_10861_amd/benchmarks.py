"""Benchmarks of the batched and served forms against sequential plain runs.

batched_vs_plain: the batched workload (64 runs) executed (i) one run after
another with the plain API on one stream, (ii) as one pool with batched
launches, its launch shape tuned online.  Aggregate agent-replications/s of
each.

served_vs_plain: the served request list replayed in real time (i) through
the continuous-batching server (serve.py), (ii) through a plain server that
runs one request at a time in arrival order.  Aggregate replications/s and
p50/p99 latency from arrival to the MRCA result on the host.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import autotune
from . import binding as hs
from . import serve as srv


def _arena_for(cfgs, gens, dev):
    need = max(hs.footprint_bytes(c, gens) for c in cfgs)
    buf = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    off = (-buf.data_ptr()) % 256
    return buf, buf[off:off + need]


def small_run(spec, dev, stream, repeats: int = 5) -> dict:
    """A run too small to fill the chip (the CPU-scale workload), timed
    whole: plain ga_step launches, and the same run as a one-run pool whose
    generations replay from a captured hipGraph.  Returns the rates and the
    plain run's final records (host copies) for comparison."""
    cfg = hs.Config(**spec.config_kwargs())
    best, kern = float("inf"), 0.0
    final = None
    for k in range(repeats + 1):
        run = hs.Run(cfg, max_gens_per_launch=spec.generations, device=dev, stream=stream)
        run.set_kernel_timing(k > 0)
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        run.step(spec.generations)
        run.sync()
        dt = time.perf_counter() - t0
        if k > 0:                           # the first run warms the process up
            best = min(best, dt)
            ms, n = run.kernel_time()
            kern = ms * 1000.0 / max(n, 1)
        if k == repeats:
            final = [np.array(x, copy=True) for x in run.agents()]
        run.close()
    pooled = batched_vs_plain([spec], dev, stream, tune=False, block_threads=64)
    return {
        "workload": spec.name,
        "replications_per_s": spec.replications / best,
        "wall_s": best,
        "us_per_generation": best * 1e6 / spec.generations,
        "step_kernel_avg_us": kern,
        "as_one_run_pool_with_graph_replay": {
            k: pooled[k] for k in ("batched_s", "batched_replications_per_s", "tuned")},
        "_final": final,
    }


def batched_vs_plain(specs, dev, stream, gens_per_launch: int = 512, tune: bool = True,
                     block_threads: int = 256) -> dict:
    cfgs = [hs.Config(**s.config_kwargs()) for s in specs]
    reps = sum(s.replications for s in specs)
    # (i) sequential plain runs, one arena reused in stream order
    gmax = max(s.generations for s in specs)
    _keep, arena = _arena_for(cfgs, gmax, dev)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for s, c in zip(specs, cfgs):
        run = hs.Run(c, max_gens_per_launch=gmax, device=dev, stream=stream, arena=arena)
        run.step(s.generations)
        run.close()
    torch.cuda.synchronize(dev)
    t_plain = time.perf_counter() - t0
    del _keep, arena
    # (ii) one pool, batched launches
    pstream = torch.cuda.Stream(dev)
    probe = hs.Pool(1 << 20, max_runs=1, max_gens_per_launch=gens_per_launch, device=dev,
                    stream=pstream)
    total = sum(probe.footprint(c) for c in cfgs)
    probe.close()
    pool = hs.Pool(total + hs.pool_overhead_bytes(len(specs)) + (1 << 20), max_runs=len(specs),
                   max_gens_per_launch=gens_per_launch, device=dev, stream=pstream)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for s, c in zip(specs, cfgs):
        if pool.admit(c, s.generations) is None:
            raise RuntimeError("pool sized too small")
    choice = {"block_threads": block_threads, "gens_per_launch": 64, "use_graph": True}
    if tune:
        choice = autotune.tune_online(pool, key=autotune.signature(specs), use_cache=False)
    else:
        pool.set_launch(block_threads, True)
    G = choice["gens_per_launch"]
    # the generations after tuning, timed on the pool's stream: wall time
    # per generation of every run, the groups' launches side by side
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    steady = 0
    e0.record(pstream)
    while True:
        n = pool.advance(G)
        if not n:
            break
        steady += n
    e1.record(pstream)
    pool.sync()
    t_batch = time.perf_counter() - t0
    done = pool.poll()
    ok = len(done) == len(specs) and all(pool.run(i).generation == specs[i].generations
                                         for i in range(len(specs)))
    pool.close()
    return {
        "workload": f"{len(specs)} runs, {reps:,} agent-replications",
        "replications": reps,
        "plain_sequential_s": t_plain,
        "plain_sequential_replications_per_s": reps / t_plain,
        "batched_s": t_batch,
        "batched_replications_per_s": reps / t_batch,
        "batched_over_plain": t_plain / t_batch,
        "steady_generations": steady,
        "steady_generation_us": e0.elapsed_time(e1) * 1000.0 / steady if steady else None,
        "tuned": {k: choice[k] for k in ("block_threads", "gens_per_launch", "use_graph")},
        "tuner_trials": choice.get("trials", []),
        "all_runs_finished": bool(ok),
    }


def plain_fifo_server(reqs, dev, stream, sample: int = 1024, time_scale: float = 1.0,
                      progress=None) -> dict:
    """One request at a time, in arrival order, with the plain API."""
    order = sorted(range(len(reqs)), key=lambda i: reqs[i].arrival)
    cfgs = {i: hs.Config(**reqs[i].config_kwargs()) for i in order}
    gmax = max(r.generations for r in reqs)
    _keep, arena = _arena_for(list(cfgs.values()), gmax, dev)
    ws = hs.MrcaWorkspace(64, sample, dev)
    lb = torch.empty((sample, sample), dtype=torch.int32, device=dev)
    ub = torch.empty((sample, sample), dtype=torch.int32, device=dev)
    lat = []
    t0 = time.perf_counter()
    next_note = 10.0
    with torch.cuda.stream(stream):
        for i in order:
            if progress is not None and time.perf_counter() - t0 >= next_note:
                progress(f"plain t={time.perf_counter() - t0:.0f}s done={len(lat)}")
                next_note += 10.0
            r = reqs[i]
            arr = r.arrival * time_scale
            now = time.perf_counter() - t0
            if now < arr:
                time.sleep(arr - now)
            run = hs.Run(cfgs[i], max_gens_per_launch=gmax, device=dev, stream=stream,
                         arena=arena)
            run.step(r.generations)
            _, cnt, srf = run.sample(sample)
            n = cnt.shape[0]
            lv = lb[:n, :n] if n == sample else torch.empty((n, n), dtype=torch.int32, device=dev)
            uv = ub[:n, :n] if n == sample else torch.empty((n, n), dtype=torch.int32, device=dev)
            run.mrca_bounds(cnt, srf, workspace=ws, lb=lv, ub=uv)
            lv.cpu()
            uv.cpu()
            run.close()
            lat.append(time.perf_counter() - t0 - arr)
    wall = time.perf_counter() - t0
    reps = sum(r.replications for r in reqs)
    lat = np.array(lat)
    return {"wall_s": wall, "replications_per_s": reps / wall,
            "latency_p50_s": float(np.percentile(lat, 50)),
            "latency_p99_s": float(np.percentile(lat, 99)),
            "latency_max_s": float(lat.max())}


def served_vs_plain(reqs, dev, chunk_gens: int = 256, time_scale: float = 1.0,
                    pool_bytes: int = 16 << 30, plain: bool = True, progress=None) -> dict:
    pstream = torch.cuda.Stream(dev)
    pool = hs.Pool(pool_bytes, max_runs=256, max_gens_per_launch=chunk_gens, device=dev,
                   stream=pstream, block_threads=64, use_graph=False)
    rep = srv.serve(pool, reqs, chunk_gens=chunk_gens, sample=1024, time_scale=time_scale,
                    progress=progress)
    pool.close()
    out = {
        "requests": len(reqs),
        "time_scale": time_scale,
        "offered_replications_per_s": sum(r.replications for r in reqs) /
                                      (max(r.arrival for r in reqs) * time_scale),
        "served": rep.summary(),
    }
    if plain:
        out["plain_fifo"] = plain_fifo_server(reqs, dev, torch.cuda.Stream(dev),
                                              time_scale=time_scale, progress=progress)
        out["served_over_plain_throughput"] = (out["served"]["replications_per_s"] /
                                               out["plain_fifo"]["replications_per_s"])
    return out


def treatment_pair(specs, dev, stream, n_sample: int = 4096, labels=None,
                   allpairs: bool = True, progress=None, keep_samples: bool = False) -> dict:
    """A treatment pair: each run, its stratified sample, all-pairs MRCA
    bounds (if allpairs) and the reconstructed tree's phylometrics (sum
    branch length, mean evolutionary distinctiveness, mean pairwise
    distance).  Integer pair (selection, neutral): selection sweeps make
    common ancestry more recent.  Float trial (purifying-only,
    adaptation-enabled): the purifying-only tree is the longer one."""
    if labels is None:
        labels = ["selection" if s.tournament_size == 2 else "neutral" for s in specs]
    out = {}
    ws = hs.MrcaWorkspace(max(s.surface_sites for s in specs), n_sample, dev) if allpairs else None
    lb = torch.empty((n_sample, n_sample), dtype=torch.int32, device=dev) if allpairs else None
    ub = torch.empty((n_sample, n_sample), dtype=torch.int32, device=dev) if allpairs else None
    for s, label in zip(specs, labels):
        if progress is not None:
            progress(f"{label}: {s.name}, {s.generations} generations")
        cfg = hs.Config(**s.config_kwargs())
        run = hs.Run(cfg, max_gens_per_launch=min(s.generations, 4096), device=dev,
                     stream=stream)
        run.set_kernel_timing(True)
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        run.step(s.generations)
        _, cnt, srf = run.sample(n_sample)
        if not out:
            # first queries of the process: workspace and table set-up
            # outside the timed queries (latencies are steady-state)
            if allpairs:
                run.mrca_bounds(cnt, srf, workspace=ws, lb=lb, ub=ub)
            run.phylo_tree(cnt, srf, tree=False)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e2 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        if allpairs:
            run.mrca_bounds(cnt, srf, workspace=ws, lb=lb, ub=ub)
        e1.record(stream)
        phylo = run.phylo_tree(cnt, srf, tree=False)
        e2.record(stream)
        torch.cuda.synchronize(dev)
        wall = time.perf_counter() - t0
        ms, launches = run.kernel_time()
        trait = run.agents(0, 65536)[0]
        if keep_samples:
            # host copies of the sample, under a key the caller removes
            out.setdefault("_samples", {})[label] = (hs.as_u32(cnt), hs.as_u32(srf))
        rec = {
            "workload": s.name,
            "replications_per_s": s.replications / wall,
            "wall_s": wall,
            "step_kernel_avg_us": ms * 1000.0 / max(launches, 1),
            "sample": int(cnt.shape[0]),
            "phylo_ms": e1.elapsed_time(e2),
            "sum_branch_length": phylo["sum_branch_length"],
            "mean_evolutionary_distinctiveness": phylo["mean_ed"],
            "mean_pairwise_distance": phylo["mean_pairwise_distance"],
            "root_time": phylo["root_time"],
            "internal_nodes": phylo["internal_nodes"],
        }
        if s.fitness_model == "float":
            rec["mean_fitness_first_65536"] = float(trait.view(np.float32).mean())
        else:
            rec["mean_trait_first_65536"] = float(trait.view(np.int32).mean())
        if allpairs:
            l_h = hs.as_u32(lb).astype(np.float64)
            u_h = hs.as_u32(ub).astype(np.float64)
            off = ~np.eye(n_sample, dtype=bool)
            rec.update({"mrca_query_ms": e0.elapsed_time(e1), "mrca_pairs": n_sample * n_sample,
                        "mean_lb": float(l_h[off].mean()), "mean_ub": float(u_h[off].mean())})
            # the same query without the run: the layout from the site rule's
            # tables (uploaded into the workspace by the call); same bounds
            lb2, ub2 = torch.empty_like(lb), torch.empty_like(ub)
            e3 = torch.cuda.Event(enable_timing=True)
            e4 = torch.cuda.Event(enable_timing=True)
            e3.record(stream)
            hs.mrca_bounds(cfg.surface_kind, cfg.surface_sites, cnt, srf, workspace=ws,
                           stream=stream, lb=lb2, ub=ub2, bits=cfg.differentia_bits,
                           interval=cfg.ingest_interval)
            e4.record(stream)
            torch.cuda.synchronize(dev)
            rec["mrca_query_from_rule_ms"] = e3.elapsed_time(e4)
            rec["mrca_query_from_rule_equal"] = bool(torch.equal(lb, lb2) and torch.equal(ub, ub2))
            del lb2, ub2
        out[label] = rec
        run.close()
    return out


def clade_trial(specs, dev, stream) -> dict:
    """The clade trial: for each duration, the founding clades still
    present, the mean MRCA bounds of same-clade and different-clade pairs
    over the whole population, and the tree of one agent sampled per
    island (its clade labels listed in sample order)."""
    out = {}
    for s in specs:
        cfg = hs.Config(**s.config_kwargs())
        run = hs.Run(cfg, device=dev, stream=stream)
        run.step(s.generations)
        tags, cnt, srf = run.agents()
        c_d = torch.from_numpy(cnt.view(np.int32)).to(dev)
        s_d = torch.from_numpy(srf.view(np.int32)).to(dev)
        lb, ub = hs.mrca_bounds(s.surface_kind, s.surface_sites, c_d, s_d, stream=stream)
        ub_h = hs.as_u32(ub).astype(np.float64)
        same = tags[:, None] == tags[None, :]
        off = ~np.eye(len(tags), dtype=bool)
        # one agent per island, as in the paper's reconstructions
        pick = np.arange(cfg.islands) * cfg.pop_per_island
        tree = hs.phylo_metrics(s.surface_kind, s.surface_sites, c_d[pick], s_d[pick],
                                stream=stream)
        out[str(s.generations)] = {
            "clades_remaining": int(len(np.unique(tags))),
            "mean_ub_same_clade": float(ub_h[same & off].mean()) if (same & off).any() else None,
            "mean_ub_different_clades": float(ub_h[~same].mean()) if (~same).any() else None,
            "per_island_sample_tags": [int(t) for t in tags[pick]],
            "per_island_tree": {k: tree[k] for k in ("sum_branch_length", "root_time",
                                                     "internal_nodes")},
        }
        run.close()
    return out


def async_vs_sync(spec, activity: float, dev, stream) -> dict:
    """The paper-scale torus run in asynchronous ticks (each island active
    with probability `activity` per tick) against the same run in
    synchronous generations: agent-ticks per second, the step kernel's
    average time, and how far the islands drift apart."""
    out = {}
    for mode in ("synchronous", "asynchronous"):
        kw = spec.config_kwargs()
        if mode == "asynchronous":
            kw["async_activity"] = int(activity * 2**32)
        cfg = hs.Config(**kw)
        run = hs.Run(cfg, max_gens_per_launch=spec.generations, device=dev, stream=stream)
        run.set_kernel_timing(True)
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        run.step(spec.generations)
        run.sync()
        wall = time.perf_counter() - t0
        ms, launches = run.kernel_time()
        counters = run.agents(0, min(cfg.agents, 1 << 20))[1]
        out[mode] = {
            "agent_ticks_per_s": cfg.agents * spec.generations / wall,
            "expected_births_per_s": cfg.agents * spec.generations *
                                     (activity if mode == "asynchronous" else 1.0) / wall,
            "wall_s": wall,
            "step_kernel_avg_us": ms * 1000.0 / max(launches, 1),
            "counter_min": int(counters.min()), "counter_max": int(counters.max()),
            "counter_mean": float(counters.mean()),
        }
        # the end-of-run query on a 4,096-agent sample: with drifted
        # counters the annotations differ in age, so every pair takes the
        # general route (per-annotation layouts, merged time lists)
        n = 4096
        _, cnt, srf = run.sample(n)
        ws = hs.MrcaWorkspace(spec.surface_sites, n, dev)
        lb = torch.empty((n, n), dtype=torch.int32, device=dev)
        ub = torch.empty((n, n), dtype=torch.int32, device=dev)
        run.mrca_bounds(cnt, srf, workspace=ws, lb=lb, ub=ub)      # warm-up
        torch.cuda.synchronize(dev)
        best = float("inf")
        for _ in range(3):
            t0 = time.perf_counter()
            run.mrca_bounds(cnt, srf, workspace=ws, lb=lb, ub=ub)
            torch.cuda.synchronize(dev)
            best = min(best, time.perf_counter() - t0)
        out[mode]["mrca_query_ms"] = best * 1e3
        out[mode]["mrca_pairs_per_s"] = n * n / best
        out[mode]["sample_counters_distinct"] = int(len(np.unique(hs.as_u32(cnt))))
        run.close()
    out["activity"] = activity
    out["ticks"] = spec.generations
    return out
