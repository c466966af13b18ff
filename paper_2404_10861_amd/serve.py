"""Served runs: continuous batching of GA runs on one GPU.

Requests (workloads.RunSpec with an arrival time) are admitted to a Pool in
arrival order as soon as their HBM footprint fits; every admitted run
advances together in chunks of generations (one batched launch per
generation); a finished run is sampled, its all-pairs MRCA bounds are
computed on the device and copied to the host, and its memory is
released.  Latency is measured from arrival to the result on the host.

The arithmetic of a run does not depend on what else is in the pool: each
result equals the same request run alone.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import binding as hs


@dataclass
class Served:
    index: int
    arrival: float
    admitted: float = 0.0
    done: float = 0.0
    replications: int = 0
    lb: np.ndarray | None = None
    ub: np.ndarray | None = None
    sample_idx: np.ndarray | None = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class ServeReport:
    results: list = field(default_factory=list)
    wall: float = 0.0
    advances: int = 0
    refused_admissions: int = 0
    peak_active: int = 0
    agents: dict = field(default_factory=dict)

    def latencies(self):
        return np.array([r.latency for r in self.results])

    def summary(self) -> dict:
        lat = self.latencies()
        reps = sum(r.replications for r in self.results)
        return {
            "requests": len(self.results),
            "wall_s": self.wall,
            "replications": reps,
            "replications_per_s": reps / self.wall if self.wall else 0.0,
            "latency_p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
            "latency_p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
            "latency_max_s": float(lat.max()) if len(lat) else None,
            "advances": self.advances,
            "refused_admissions": self.refused_admissions,
            "peak_active": self.peak_active,
        }


def run_alone(spec, sample: int = 1024, device="cuda", stream=None):
    """The same request on its own through the plain API: (agents, lb, ub)."""
    cfg = hs.Config(**spec.config_kwargs())
    run = hs.Run(cfg, device=device, stream=stream)
    run.step(spec.generations)
    idx, cnt, srf = run.sample(sample)
    lb, ub = hs.mrca_bounds(spec.surface_kind, spec.surface_sites, cnt, srf, stream=stream,
                            bits=spec.differentia_bits, interval=spec.ingest_interval)
    out = (run.agents(), hs.as_u32(idx), hs.as_u32(lb), hs.as_u32(ub))
    run.close()
    return out


def serve(pool: hs.Pool, requests, chunk_gens: int = 256, sample: int = 1024,
          keep_results: bool = False, time_scale: float = 1.0, keep_agents=None,
          progress=None) -> ServeReport:
    """Serve `requests` (sorted or not) in real time.

    time_scale stretches (>1) or compresses (<1) the arrival times.
    keep_results keeps each run's lb/ub matrices and sample indices on the
    host; keep_agents (a set of request indices) also keeps their final
    records in `report.agents`.  progress(text), if given, is called about
    every 10 s with the loop's state.
    """
    dev = pool.device
    stream = pool.stream
    ws = hs.MrcaWorkspace(64, sample, dev)
    lb_dev = torch.empty((sample, sample), dtype=torch.int32, device=dev)
    ub_dev = torch.empty((sample, sample), dtype=torch.int32, device=dev)
    idx_buf = torch.empty(sample, dtype=torch.int32, device=dev)
    cnt_buf = torch.empty(sample, dtype=torch.int32, device=dev)
    srf_buf = {1: torch.empty((sample, 1), dtype=torch.int32, device=dev),
               2: torch.empty((sample, 2), dtype=torch.int32, device=dev)}
    reqs = sorted(enumerate(requests), key=lambda x: x[1].arrival)
    pending = deque(reqs)
    waiting: deque = deque()
    active: dict[int, tuple] = {}
    report = ServeReport()
    keep_agents = keep_agents or set()
    t0 = time.perf_counter()
    next_note = 10.0
    while pending or waiting or active:
        now = time.perf_counter() - t0
        if progress is not None and now >= next_note:
            progress(f"served t={now:.0f}s done={len(report.results)} active={len(active)} "
                     f"waiting={len(waiting)} pending={len(pending)}")
            next_note += 10.0
        while pending and pending[0][1].arrival * time_scale <= now:
            i, spec = pending.popleft()
            waiting.append((i, spec, spec.arrival * time_scale))
        while waiting:
            i, spec, arr = waiting[0]
            rid = pool.admit(hs.Config(**spec.config_kwargs()), spec.generations)
            if rid is None:
                report.refused_admissions += 1
                break
            waiting.popleft()
            active[rid] = (i, spec, arr, time.perf_counter() - t0)
        report.peak_active = max(report.peak_active, len(active))
        if not active:
            if pending:
                delay = pending[0][1].arrival * time_scale - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(delay)
                continue
            if waiting:
                raise RuntimeError("a request does not fit in an empty pool")
            break
        pool.advance(chunk_gens)
        report.advances += 1
        finished = pool.poll()
        with torch.cuda.stream(stream):
            for rid in finished:
                i, spec, arr, adm = active[rid]
                run = pool.run(rid)
                sw = spec.surface_sites * spec.differentia_bits // 32
                idx, cnt, srf = run.sample(sample, out=(idx_buf, cnt_buf, srf_buf[sw]))
                n = cnt.shape[0]
                lb_v = lb_dev[:n, :n] if n == sample else torch.empty((n, n), dtype=torch.int32,
                                                                       device=dev)
                ub_v = ub_dev[:n, :n] if n == sample else torch.empty((n, n), dtype=torch.int32,
                                                                       device=dev)
                run.mrca_bounds(cnt, srf, workspace=ws, lb=lb_v, ub=ub_v)
                lb_h = lb_v.to("cpu", non_blocking=False)
                ub_h = ub_v.to("cpu", non_blocking=False)
                res = Served(index=i, arrival=arr, admitted=adm,
                             replications=spec.agents * spec.generations)
                if keep_results:
                    res.lb = lb_h.numpy().view(np.uint32)
                    res.ub = ub_h.numpy().view(np.uint32)
                    res.sample_idx = hs.as_u32(idx)
                if i in keep_agents:
                    report.agents[i] = run.agents()
                res.done = time.perf_counter() - t0
                report.results.append(res)
                pool.release(rid)
                del active[rid]
    report.wall = time.perf_counter() - t0
    report.results.sort(key=lambda r: r.index)
    return report
