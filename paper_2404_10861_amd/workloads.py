"""The five synthetic workloads, as seeded generators of run configurations.

This module holds none of the method's arithmetic: it only states the
configurations (torus, agents per island, surface kind and size, selection,
mutation, generation counts, seeds) and draws the batched and served run
sets from numpy's seeded generator.  The paper's workloads are themselves
synthetic simulations; there is no dataset to stand in for.

* C1 plain, CPU-scale: 8x8 islands x 32 agents, 32-site steady, 1,000 gens.
* C2 plain, paper-scale: 512x1024 islands x 32 agents (16.8 M agents),
  64-site hybrid, 10,000 generations.
* C3 treatment pair: 256x256 islands x 64 agents (4.2 M), 32-site tilted,
  20,000 generations, tournament vs neutral; then 4,096 sampled agents and
  all-pairs MRCA bounds.
* C4 batched: 64 runs, grids from {16x16, 32x64, 64x64, 128x256}, 16/32/64
  agents per island, 32/64 sites, steady/tilted/hybrid, half selection,
  5,000 generations, seeds 1..64.
* C5 served: Poisson arrivals at 20/s over 120 s; grids log-uniform from
  8x8 to 256x512, 32 agents per island, 1,000..20,000 generations
  log-uniform, random kind and 32/64 sites; 1,024-agent MRCA at completion.
All runs: trait starts at 0, mutation p = 0.01 (threshold floor(0.01 * 2^32))
adding a uniform integer in [-8, 8], one migrant per island per generation.

* Float trial (after the paper's On-hardware Trial): 750x750 islands x 32
  agents (18 M), 64-site tilted surface (the four-word genome: binary32
  fitness, 32-bit counter, 64-bit surface), tournament of five, binary32
  fitness from 0; purifying-only (33 % of births lose del_sigma |Z|) vs
  adaptation-enabled (additionally 0.3 % gain ben_sigma |Z|), scales 1.0;
  a 10,000-agent stratified sample is reconstructed into a tree.  The
  paper ran 1,000,000 generations; the default here is 20,000.
* Clade trial (after the paper's Clade Reconstruction Trial): 3x3 islands
  x 32 agents, 64-site tilted surface, neutral selection, founder tags;
  durations 25, 50, 100 and 250 generations; one sampled agent per island
  and the whole population are reconstructed.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field

import numpy as np

MUT_THRESHOLD = 42949672   # floor(0.01 * 2^32)
P_DELETERIOUS = 1417339207  # floor(0.33 * 2^32)
P_BENEFICIAL = 12884901     # floor(0.003 * 2^32)


@dataclass
class RunSpec:
    grid_w: int
    grid_h: int
    pop_per_island: int
    surface_sites: int
    surface_kind: str
    tournament_size: int
    generations: int
    seed: int
    mut_threshold: int = MUT_THRESHOLD
    mut_lo: int = -8
    mut_hi: int = 8
    migrants_per_island: int = 1
    sample: int = 0            # agents sampled for the end-of-run MRCA query
    arrival: float = 0.0       # seconds after the start (served workload)
    name: str = ""
    fitness_model: str = "int"
    del_threshold: int = 0
    ben_threshold: int = 0
    del_sigma: float = 1.0
    ben_sigma: float = 1.0
    differentia_bits: int = 1
    ingest_interval: int = 1

    @property
    def agents(self) -> int:
        return self.grid_w * self.grid_h * self.pop_per_island

    @property
    def replications(self) -> int:
        return self.agents * self.generations

    def config_kwargs(self) -> dict:
        return dict(grid_w=self.grid_w, grid_h=self.grid_h, pop_per_island=self.pop_per_island,
                    surface_sites=self.surface_sites, surface_kind=self.surface_kind,
                    tournament_size=self.tournament_size, mut_threshold=self.mut_threshold,
                    mut_lo=self.mut_lo, mut_hi=self.mut_hi,
                    migrants_per_island=self.migrants_per_island, seed=self.seed,
                    fitness_model=self.fitness_model, del_threshold=self.del_threshold,
                    ben_threshold=self.ben_threshold, del_sigma=self.del_sigma,
                    ben_sigma=self.ben_sigma, differentia_bits=self.differentia_bits,
                    ingest_interval=self.ingest_interval)


def c1() -> RunSpec:
    return RunSpec(8, 8, 32, 32, "steady", 2, 1000, seed=1, name="C1 plain 8x8x32 steady-32")


def c2() -> RunSpec:
    return RunSpec(512, 1024, 32, 64, "hybrid", 2, 10000, seed=1,
                   name="C2 plain 512x1024x32 hybrid-64")


def c3(selection: bool) -> RunSpec:
    return RunSpec(256, 256, 64, 32, "tilted", 2 if selection else 0, 20000, seed=1, sample=4096,
                   name=f"C3 {'selection' if selection else 'neutral'} 256x256x64 tilted-32")


def trial(adaptive: bool, side: int = 750, generations: int = 20000) -> RunSpec:
    """One treatment of the float trial (purifying-only or adaptation-enabled)."""
    name = "adaptation-enabled" if adaptive else "purifying-only"
    return RunSpec(side, side, 32, 64, "tilted", 5, generations, seed=1, sample=10000,
                   fitness_model="float", del_threshold=P_DELETERIOUS,
                   ben_threshold=P_BENEFICIAL if adaptive else 0,
                   name=f"float trial {name} {side}x{side}x32 tilted-64")


def clade(generations: int, seed: int = 17) -> RunSpec:
    """The clade trial (after the paper's Clade Reconstruction Trial): 3x3
    islands x 32 agents, 64-site tilted surface, neutral selection, random
    16-bit founder tags inherited without mutation."""
    return RunSpec(3, 3, 32, 64, "tilted", 0, generations, seed=seed, fitness_model="tag",
                   name=f"clade trial 3x3x32 tilted-64, {generations} generations")


C4_GRIDS = ((16, 16), (32, 64), (64, 64), (128, 256))
C4_POPS = (16, 32, 64)
C4_SITES = (32, 64)
C4_KINDS = ("steady", "tilted", "hybrid")


def c4(draw_seed: int = 20240417) -> list[RunSpec]:
    """64 replicate runs; run r (1..64) has seed r, selection iff r <= 32."""
    rng = np.random.default_rng(draw_seed)
    runs = []
    for r in range(1, 65):
        gw, gh = C4_GRIDS[int(rng.integers(len(C4_GRIDS)))]
        n = C4_POPS[int(rng.integers(len(C4_POPS)))]
        s = C4_SITES[int(rng.integers(len(C4_SITES)))]
        k = C4_KINDS[int(rng.integers(len(C4_KINDS)))]
        runs.append(RunSpec(gw, gh, n, s, k, 2 if r <= 32 else 0, 5000, seed=r,
                            name=f"C4 run {r}"))
    return runs


def c5(duration: float = 120.0, rate: float = 20.0, draw_seed: int = 20240418) -> list[RunSpec]:
    """Served request list: exponential inter-arrival times (mean 1/rate)."""
    rng = np.random.default_rng(draw_seed)
    reqs = []
    t = 0.0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        w = int(round(2.0 ** (3 + 5 * rng.random())))       # 8 .. 256
        h = int(round(2.0 ** (3 + 6 * rng.random())))       # 8 .. 512
        g = int(round(1000 * 20.0 ** rng.random()))         # 1,000 .. 20,000
        kind = C4_KINDS[int(rng.integers(3))]
        s = C4_SITES[int(rng.integers(2))]
        idx = len(reqs)
        reqs.append(RunSpec(w, h, 32, s, kind, 2, g, seed=idx + 1, sample=1024, arrival=t,
                            name=f"C5 request {idx}"))
    return reqs


# The batched and served run sets as saved lists (data/, written once by
# make_workload_lists.py from c4() and c5()): the lists, not the draws, are
# the workloads, so they do not depend on numpy's generator staying the same.
DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")
C4_LIST = os.path.join(DATA, "c4_runs.json")
C5_LIST = os.path.join(DATA, "c5_requests.json")


def c4_rows(runs: list[RunSpec]) -> list:
    return [[r.grid_w, r.grid_h, r.pop_per_island, r.surface_sites, r.surface_kind,
             r.tournament_size, r.generations, r.seed] for r in runs]


def c5_rows(reqs: list[RunSpec]) -> list:
    return [[round(r.arrival, 9), r.grid_w, r.grid_h, r.generations, r.surface_kind,
             r.surface_sites, r.seed] for r in reqs]


def c4_saved() -> list[RunSpec]:
    """The 64-run batched set as saved."""
    with open(C4_LIST) as f:
        rows = json.load(f)["runs"]
    return [RunSpec(w, h, n, s, k, t, g, seed=sd, name=f"C4 run {sd}")
            for w, h, n, s, k, t, g, sd in rows]


def c5_saved(duration: float = 120.0) -> list[RunSpec]:
    """The served request list as saved (arrivals before `duration` s)."""
    with open(C5_LIST) as f:
        rows = json.load(f)["requests"]
    return [RunSpec(w, h, 32, s, k, 2, g, seed=sd, sample=1024, arrival=a,
                    name=f"C5 request {sd - 1}")
            for a, w, h, g, k, s, sd in rows if a < duration]


def offered_replication_rate(reqs: list[RunSpec], duration: float) -> float:
    return sum(r.replications for r in reqs) / duration


def log_uniform_check(values, lo, hi) -> bool:
    """Every value within [lo, hi] (used by tests of the generators)."""
    return all(lo <= v <= hi for v in values) and not math.isnan(sum(values))
