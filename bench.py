"""Benchmark of the island-model GA hot path on one MI355X.

One "step" is one whole run of the paper-scale plain workload: 512x1024
islands x 32 agents (16.8 M agents), 64-site hybrid surface, tournament of
two, mutation p = 0.01 in [-8, 8], one migrant per island per generation,
10,000 generations; then a stratified 4,096-agent sample and its all-pairs
MRCA-generation bounds (16.8 M pairs).  Inputs are synthetic (the founders
are generated on the device; the paper's workloads are synthetic too).

Prints one JSON line:
  value     agent-replications/s over the timed steps (births only)
  roofline  the step kernel's algorithmic HBM bytes per launch (what a
            synchronous generation must move) over its average launch
            duration (HIP events on the run's stream);
            traffic: the HBM bytes per launch that rocprofv3 counted for
            the same code (profiles/), null once the code has changed
  cpu_baseline  the plain C oracle on a bounded sample of the same
            workload (the first generations from the founders).

  batched_vs_plain  the rest of the metric, measured after the timed
            steps: the 64-run batched workload against the same runs one
            at a time, and a window of the served workload's arrivals
            against a one-at-a-time server, with p50/p99 run latency
            (skipped with --no-pools or when --generations is given).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       [--generations G] [--no-cpu-baseline] [--no-pools]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_c2_traffic.json")
SQ_FILE = os.path.join(ROOT, "profiles", "step_kernel_c2_sq_counters.json")


def algorithmic_bytes_per_generation(spec) -> int:
    """The bytes one synchronous generation has to move: the trait and
    surface words of every parent read and of every child written (a
    record of 4 + S/8 bytes: every counter is the generation number, so
    none is stored), and each island's 16-byte migrant entry (direction,
    trait, surface words) written once and read once."""
    rec = 4 + spec.surface_sites // 8
    islands = spec.grid_w * spec.grid_h
    return 2 * spec.agents * rec + 2 * islands * 16


def record_model_bytes_per_generation(spec) -> int:
    """The same generation priced with a stored 32-bit counter in every
    record (8 + S/8 bytes) and a 32-byte migrant entry per island: what a
    design that keeps per-agent counters would move (asynchronous ticks
    do)."""
    rec = 8 + spec.surface_sites // 8
    islands = spec.grid_w * spec.grid_h
    return 2 * spec.agents * rec + islands * 32


def batch_bytes_per_generation(spec) -> int:
    """algorithmic_bytes_per_generation for any run of a batch (migrant
    entries only when migration is on)."""
    rec = 4 + spec.surface_sites * spec.differentia_bits // 8
    islands = spec.grid_w * spec.grid_h
    return 2 * spec.agents * rec + (2 * islands * 16 if spec.migrants_per_island else 0)


def measured_traffic(spec):
    """HBM bytes per step launch from the committed rocprofv3 counter
    summary, or None when it is absent or the kernel changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        rec = json.load(f)
    from paper_2404_10861_amd.profiling import kernel_hash
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


def measured_valu():
    """The step kernel's VALU figures from the committed rocprofv3 SQ
    counter summary, or None when it is absent or the kernel changed since."""
    if not os.path.exists(SQ_FILE):
        return None
    with open(SQ_FILE) as f:
        rec = json.load(f)
    from paper_2404_10861_amd.profiling import kernel_hash
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return {"issue_estimate": rec["valu_issue_estimate"],
            "instructions_per_wave": rec["valu_instructions_per_wave"],
            "resident_waves_per_simd": rec["resident_waves_per_simd"],
            "wave_time_waiting": rec["wave_time_waiting"],
            "source": "profiles/step_kernel_c2_sq_counters.json (rocprofv3 SQ counters; "
                      "issue estimate counts 4 cycles per VALU instruction)"}


def attainable_copy_gbs(torch, hs, dev, stream, nbytes: int = 512 << 20, reps: int = 10):
    """Bandwidth of the library's plain 16-byte copy kernel over buffers
    larger than the 256 MB Infinity Cache (read + write bytes / time)."""
    src = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    dst = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    src.fill_(1)
    hs.probe_copy(src, dst, stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        hs.probe_copy(src, dst, stream)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * nbytes / (ms / 1000.0) / 1e9


def host_cpu() -> dict:
    """The host's CPU model, its logical CPU count and the CPUs this process
    may run on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"cpu_model": model or "unknown", "nproc": os.cpu_count() or 1,
            "usable_cpus": usable}


def _oracle_rate(orc, spec, threads: int, budget_s: float, max_gens: int = 200) -> tuple:
    """Births per second of the oracle on the first generations of `spec`
    from the founders, stopping once the budget is spent."""
    r = orc.Run(spec.grid_w, spec.grid_h, spec.pop_per_island, spec.surface_sites,
                orc.KINDS[spec.surface_kind], spec.tournament_size, spec.mut_threshold,
                spec.mut_lo, spec.mut_hi, spec.migrants_per_island, spec.seed, threads=threads)
    gens = 0
    t0 = time.perf_counter()
    while True:
        r.step(1)
        gens += 1
        el = time.perf_counter() - t0
        if el >= budget_s or gens >= max_gens:
            break
    r.close()
    return spec.agents * gens / el, gens, el


def cpu_baseline(spec, budget_s: float = 6.0):
    """The oracle on the host's cores: island-parallel on the CPUs this
    process may use (at most 16) and single-threaded, each
    on the first generations of the paper-scale workload; plus bounded
    prefixes of the treatment-pair and batched workloads, extrapolated to
    their full lengths and labelled so."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import hsga_oracle as orc
    if not os.path.exists(orc.LIB):
        orc.build()
    from paper_2404_10861_amd import workloads as wl
    cpu = host_cpu()
    threads = max(1, min(16, cpu["usable_cpus"]))
    rate_t, gens_t, el_t = _oracle_rate(orc, spec, threads, budget_s)
    rate_1, gens_1, el_1 = _oracle_rate(orc, spec, 1, budget_s)
    # the treatment pair's selection run and the 64 batched runs: a few
    # generations each on all threads, extrapolated
    c3 = wl.c3(True)
    rate_c3, gens_c3, _ = _oracle_rate(orc, c3, threads, 2.0)
    c4 = wl.c4_saved()
    t0 = time.perf_counter()
    c4_births = 0
    for sp in c4:
        r = orc.Run(sp.grid_w, sp.grid_h, sp.pop_per_island, sp.surface_sites,
                    orc.KINDS[sp.surface_kind], sp.tournament_size, seed=sp.seed,
                    threads=threads)
        r.step(2)
        r.close()
        c4_births += sp.agents * 2
    rate_c4 = c4_births / (time.perf_counter() - t0)
    c4_total = sum(sp.replications for sp in c4)
    return {
        "value": rate_t,
        "unit": "agent-replications/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{spec.name}: the first {gens_t} generations from the founders "
                   f"({spec.agents * gens_t:,} births in {el_t:.1f} s), plain C oracle, "
                   f"islands split over {threads} threads, one barrier per generation"),
        "single_thread": {"value": rate_1, "sample": f"the first {gens_1} generations "
                                                      f"({el_1:.1f} s), one thread"},
        **cpu,
        "other_workloads_extrapolated": {
            c3.name: {"replications_per_s": rate_c3,
                      "sample": f"the first {gens_c3} generations on {threads} threads",
                      "extrapolated_s_for_both_treatments":
                          2 * c3.replications / rate_c3},
            "C4 batched, 64 runs run one after another": {
                "replications_per_s": rate_c4,
                "sample": f"2 generations of every run on {threads} threads",
                "extrapolated_s_for_5000_generations": c4_total / rate_c4},
        },
    }


def cpu_baseline_small(spec, gpu_final):
    """The whole CPU-scale run on the oracle, single-threaded, timed; and
    whether its final records equal the GPU run's word for word."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import numpy as np
    import hsga_oracle as orc
    if not os.path.exists(orc.LIB):
        orc.build()
    r = orc.Run(spec.grid_w, spec.grid_h, spec.pop_per_island, spec.surface_sites,
                orc.KINDS[spec.surface_kind], spec.tournament_size, spec.mut_threshold,
                spec.mut_lo, spec.mut_hi, spec.migrants_per_island, spec.seed)
    t0 = time.perf_counter()
    r.step(spec.generations)
    el = time.perf_counter() - t0
    same = all(np.array_equal(np.asarray(a, np.uint32).reshape(-1),
                              np.asarray(b, np.uint32).reshape(-1))
               for a, b in zip(r.agents(), gpu_final))
    r.close()
    return {"value": spec.replications / el, "unit": "agent-replications/s", "cores": 1,
            "kind": "oracle", "sample": f"{spec.name}, the whole run ({el:.2f} s), one thread",
            **host_cpu(), "final_records_equal_gpu": bool(same)}


def cpu_baseline_query(spec, counters, surfaces, rows: int = 1024):
    """The oracle's all-pairs MRCA bounds, single-threaded, on the first
    rows of the GPU run's sample (every column), as ordered pairs per
    second."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import hsga_oracle as orc
    if not os.path.exists(orc.LIB):
        orc.build()
    import numpy as np
    n = len(counters)
    rows = min(rows, n)
    t0 = time.perf_counter()
    orc.mrca_rows(orc.KINDS[spec.surface_kind], spec.surface_sites, counters, surfaces,
                  np.arange(rows, dtype=np.uint32))
    el = time.perf_counter() - t0
    return {
        "value": rows * n / el,
        "unit": "MRCA ordered pairs/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"rows 0..{rows - 1} of the {n:,}-agent sample of {spec.name} "
                   f"({rows * n:,} ordered pairs in {el:.1f} s), plain C oracle, one thread"),
    }


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--generations", type=int, default=0,
                    help="override the run length (profiling only; not the benchmark)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", choices=("plain", "small", "batched", "served", "pair", "trial",
                                       "clade", "async"),
                    default="plain",
                    help="plain: the paper-scale run (default); batched / served: the run "
                         "sets of the batched and served workloads against sequential plain runs")
    ap.add_argument("--time-scale", type=float, default=1.0,
                    help="served mode: stretch (>1) or compress (<1) the arrival times")
    ap.add_argument("--no-plain", action="store_true",
                    help="served mode: skip the plain one-at-a-time server")
    ap.add_argument("--duration", type=float, default=120.0,
                    help="served mode: seconds of arrivals (before time scaling)")
    ap.add_argument("--no-pools", action="store_true",
                    help="plain mode: skip the batched and served summaries")
    ap.add_argument("--batch-block", type=int, default=0,
                    help="batched mode: this workgroup size instead of the autotuner's "
                         "choice (profiling)")
    ap.add_argument("--served-window", type=float, default=120.0,
                    help="plain mode: seconds of served-workload arrivals in the summary "
                         "(default: the whole 120 s request list)")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the runs are single-GPU by design)", file=sys.stderr)
        return 2

    import torch

    import paper_2404_10861_amd as hs
    from paper_2404_10861_amd import workloads as wl

    if args.mode != "plain":
        dev = torch.device("cuda:0")
        torch.cuda.set_device(dev)
        from paper_2404_10861_amd import benchmarks
        if args.mode == "small":
            spec = wl.c1()
            res = benchmarks.small_run(spec, dev, torch.cuda.current_stream(dev))
            final = res.pop("_final")
            if not args.no_cpu_baseline:
                res["cpu_baseline"] = cpu_baseline_small(spec, final)
            metric = "agent-replications/sec (CPU-scale run)"
            value = res["replications_per_s"]
        elif args.mode == "async":
            spec = wl.c2()
            spec.generations = args.generations or 2000
            res = benchmarks.async_vs_sync(spec, 0.9, dev, torch.cuda.current_stream(dev))
            metric = "agent-ticks/sec, asynchronous vs synchronous (paper-scale torus)"
            value = res["asynchronous"]["agent_ticks_per_s"]
        elif args.mode == "clade":
            t0 = time.perf_counter()
            res = benchmarks.clade_trial([wl.clade(g) for g in (25, 50, 100, 250)], dev,
                                         torch.cuda.current_stream(dev))
            metric = "clade trial: founding clades and MRCA bounds within / between clades"
            value = time.perf_counter() - t0
        elif args.mode == "trial":
            gens = args.generations or 20000
            res = benchmarks.treatment_pair(
                [wl.trial(False, generations=gens), wl.trial(True, generations=gens)], dev,
                torch.cuda.current_stream(dev), n_sample=10000,
                labels=["purifying", "adaptive"], allpairs=False,
                progress=lambda text: print(text, file=sys.stderr, flush=True))
            metric = "agent-replications/sec (float trial) and phylometrics"
            value = res["purifying"]["replications_per_s"]
        elif args.mode == "pair":
            spec_sel = wl.c3(True)
            res = benchmarks.treatment_pair([spec_sel, wl.c3(False)], dev,
                                            torch.cuda.current_stream(dev),
                                            keep_samples=not args.no_cpu_baseline)
            samples = res.pop("_samples", None)
            for label in ("selection", "neutral"):
                r = res[label]
                r["mrca_pairs_per_s"] = r["mrca_pairs"] / (r["mrca_query_ms"] / 1000.0)
            if samples is not None:
                res["cpu_baseline_query"] = cpu_baseline_query(spec_sel, *samples["selection"])
            # the same two runs as one two-run pool (batched launches): whether
            # a 4.2 M-agent generation alone leaves the chip room for another
            b = benchmarks.batched_vs_plain([spec_sel, wl.c3(False)], dev,
                                            torch.cuda.current_stream(dev))
            res["pair_as_one_pool"] = {k: b[k] for k in (
                "plain_sequential_replications_per_s", "batched_replications_per_s",
                "batched_over_plain", "tuned", "all_runs_finished")}
            metric = "agent-replications/sec (treatment pair) and MRCA query time"
            value = res["selection"]["replications_per_s"]
        elif args.mode == "batched":
            specs = wl.c4_saved()
            if args.generations:          # profiling: shorter runs of the same set
                for sp in specs:
                    sp.generations = args.generations
            stream = torch.cuda.current_stream(dev)
            copy_gbs = attainable_copy_gbs(torch, hs, dev, stream)
            res = benchmarks.batched_vs_plain(specs, dev, stream, tune=not args.batch_block,
                                              block_threads=args.batch_block or 256)
            bytes_gen = sum(batch_bytes_per_generation(sp) for sp in specs)
            res["algorithmic_bytes_per_generation"] = bytes_gen
            res["attainable_copy_GBs"] = copy_gbs
            gen_us = res["steady_generation_us"]
            if gen_us:
                gbs = bytes_gen / (gen_us * 1e-6) / 1e9
                res["roofline"] = {
                    "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": gbs / HBM_PEAK_GBS, "frac_of_attainable": gbs / copy_gbs,
                    "kernel": "batch_step_kernel, the launch groups side by side",
                    "generation_us": gen_us,
                    "note": "achieved: the set's algorithmic bytes per generation over the "
                            "wall time per generation after tuning (HIP events on the "
                            "pool's stream)"}
            metric = "agent-replications/sec (batched vs sequential plain)"
            value = res["batched_replications_per_s"]
        else:
            reqs = wl.c5_saved(duration=args.duration)
            res = benchmarks.served_vs_plain(
                reqs, dev, time_scale=args.time_scale, plain=not args.no_plain,
                progress=lambda text: print(text, file=sys.stderr, flush=True))
            metric = "agent-replications/sec and p50/p99 run latency (served)"
            value = res["served"]["replications_per_s"]
        unit = {"clade": "s (wall)", "async": "agent-ticks/s"}.get(args.mode,
                                                                   "agent-replications/s")
        print(json.dumps({"metric": metric, "value": value, "unit": unit,
                          "n_gpus": 1, "mode": args.mode,
                          "dtype": "u32,f32,f64" if args.mode == "trial" else "u32",
                          "higher_is_better": args.mode != "clade",
                          "data": "synthetic",
                          "result": res}), flush=True)
        return 0

    spec = wl.c2()
    if args.generations:
        spec.generations = args.generations
    n_sample = 4096
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    cfg = hs.Config(**spec.config_kwargs())
    gens_per_launch = spec.generations
    need = hs.footprint_bytes(cfg, gens_per_launch)
    arena = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    off = (-arena.data_ptr()) % 256
    arena_view = arena[off:off + need]
    ws = hs.MrcaWorkspace(spec.surface_sites, n_sample, dev)
    lb = torch.empty((n_sample, n_sample), dtype=torch.int32, device=dev)
    ub = torch.empty((n_sample, n_sample), dtype=torch.int32, device=dev)

    def one_run(timed: bool):
        run = hs.Run(cfg, max_gens_per_launch=gens_per_launch, device=dev, stream=stream,
                     arena=arena_view)
        run.set_kernel_timing(timed)
        run.step(spec.generations)
        _, cnt, srf = run.sample(n_sample)
        run.mrca_bounds(cnt, srf, workspace=ws, lb=lb, ub=ub)
        return run

    copy_gbs = attainable_copy_gbs(torch, hs, dev, stream)
    for _ in range(args.warmup):
        r = one_run(False)
        r.sync()
        r.close()
    torch.cuda.synchronize()
    runs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        runs.append(one_run(True))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0

    kern_ms = 0.0
    launches = 0
    for r in runs:
        ms, n = r.kernel_time()
        kern_ms += ms
        launches += n
        r.close()
    if hs.mrca_status(ws, stream) != 0:
        raise RuntimeError("MRCA query reported an error")

    reps = spec.agents * spec.generations * args.steps
    value = reps / elapsed
    bytes_per_launch = algorithmic_bytes_per_generation(spec)
    record_bytes = record_model_bytes_per_generation(spec)
    avg_launch_s = kern_ms / 1000.0 / max(launches, 1)
    achieved_gbs = bytes_per_launch / avg_launch_s / 1e9
    traffic = measured_traffic(spec)
    line = {
        "metric": "agent-replications/sec",
        "value": value,
        "unit": "agent-replications/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1000.0,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (founders generated on the device from the seed)",
        "config": {
            "workload": spec.name,
            "torus": f"{spec.grid_w}x{spec.grid_h}",
            "agents": spec.agents,
            "agents_per_island": spec.pop_per_island,
            "surface": f"{spec.surface_kind}-{spec.surface_sites}",
            "generations": spec.generations,
            "selection": "tournament-2",
            "mrca_sample": n_sample,
            "seed": spec.seed,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "step_kernel<2, kBirthIntTournament, migration, 4 agents per thread>",
            "avg_launch_us": avg_launch_s * 1e6,
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "bytes_per_replication": bytes_per_launch / spec.agents,
            "attainable_copy_GBs": copy_gbs,
            "frac_of_attainable": achieved_gbs / copy_gbs,
            "note": "algorithmic bytes: 12-byte records (trait, 64 one-bit sites; every "
                    "counter is the generation number) read and written, and one 16-byte "
                    "migrant entry written and read per island; record_model_* prices a "
                    "stored counter and 32-byte entries, which this step does not move",
            "record_model_bytes_per_launch": record_bytes,
            "record_model_GBs": record_bytes / avg_launch_s / 1e9,
            "traffic_GBs": traffic / avg_launch_s / 1e9 if traffic else None,
            "traffic_frac_of_attainable":
                traffic / avg_launch_s / 1e9 / copy_gbs if traffic else None,
            "valu": measured_valu(),
        },
        "context": {
            "paper_cs2_replications_per_s": 3.18e11,
            "paper_note": "Cerebras CS-2, 750x750 PEs x 32 agents, float genome, tournament 5",
        },
    }
    if not args.generations and not args.no_pools:
        # the rest of the metric, on the batched and served workloads
        del arena, arena_view, ws, lb, ub
        torch.cuda.synchronize(dev)
        torch.cuda.empty_cache()
        line["batched_vs_plain"] = pool_summary(torch, dev, stream, args.served_window)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(spec)
    print(json.dumps(line), flush=True)
    return 0


def pool_summary(torch, dev, stream, window_s: float) -> dict:
    """Batched and served against plain: the 64-run batched workload against
    the same runs one at a time, and a window of the served workload's
    arrivals (Poisson, 20/s, in real time) against a one-at-a-time server of
    the same requests, with p50/p99 run latency."""
    from paper_2404_10861_amd import benchmarks
    from paper_2404_10861_amd import workloads as wl
    b = benchmarks.batched_vs_plain(wl.c4_saved(), dev, stream)
    reqs = wl.c5_saved(duration=window_s)
    v = benchmarks.served_vs_plain(
        reqs, dev, progress=lambda text: print(text, file=sys.stderr, flush=True))
    return {
        "batched": {
            "workload": b["workload"],
            "replications_per_s": b["batched_replications_per_s"],
            "plain_sequential_replications_per_s": b["plain_sequential_replications_per_s"],
            "batched_over_plain": b["batched_over_plain"],
        },
        "served": {
            "workload": f"{len(reqs)} requests arriving over {window_s:g} s in real time "
                        "(Poisson, 20/s; the saved served request list)",
            "offered_replications_per_s": v["offered_replications_per_s"],
            "replications_per_s": v["served"]["replications_per_s"],
            "latency_p50_s": v["served"]["latency_p50_s"],
            "latency_p99_s": v["served"]["latency_p99_s"],
            "plain_replications_per_s": v["plain_fifo"]["replications_per_s"],
            "plain_latency_p50_s": v["plain_fifo"]["latency_p50_s"],
            "plain_latency_p99_s": v["plain_fifo"]["latency_p99_s"],
            "served_over_plain_throughput": v["served_over_plain_throughput"],
            "served_over_plain_p99_latency": v["plain_fifo"]["latency_p99_s"] /
                                             v["served"]["latency_p99_s"],
            "note": "both servers complete the offered load as it arrives, so their "
                    "throughputs over the window are the offered load (ratio near 1); the "
                    "served loop's gain at this load is latency.  Saturated arrivals "
                    "(--mode served --time-scale 0.1) measure the throughput gain",
        },
    }


if __name__ == "__main__":
    sys.exit(main())
