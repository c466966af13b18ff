"""Full-size GPU parity over many generations (about two and a half
minutes, mostly the oracle on up to 16 host threads; HSGA_SKIP_FULL=1
skips them for quick runs): the
paper-scale workload (512x1024 islands x 32, hybrid-64, tournament of two)
for 300 generations, the treatment pair's torus (256x256 x 64, tilted-32)
for 2,000 generations of each treatment, the float trial (750x750 x 32,
tilted-64, adaptation-enabled) for 100 generations, and asynchronous ticks on
the paper-scale torus (activity 0.9) for 200 ticks: every agent word, the
layout and every outbox entry against the oracle, in the launch
configuration the benchmarks use; for the integer runs also every pair of
the benchmark's 4,096-agent MRCA query and its reconstructed tree."""
import os
import sys
import time

import numpy as np
import pytest

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(os.environ.get("HSGA_SKIP_FULL") == "1",
                                 reason="HSGA_SKIP_FULL=1")]


@pytest.fixture(scope="module")
def hs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_10861_amd as hs
    hs.load_library()
    return hs


# the oracle's island-parallel mode for synchronous runs (the same words
# as one thread; asynchronous ticks stay serial)
THREADS = min(16, os.cpu_count() or 1)


def oracle_steps(o, G, label):
    """Step the oracle G generations, printing progress now and then."""
    t0 = time.perf_counter()
    done = 0
    while done < G:
        k = min(50, G - done)
        o.step(k)
        done += k
        print(f"{label}: oracle at generation {done} ({time.perf_counter() - t0:.0f} s)",
              file=sys.stderr, flush=True)


@pytest.mark.parametrize("W,H,N,S,kind,tour,G", [
    (512, 1024, 32, 64, "hybrid", 2, 300),
    (256, 256, 64, 32, "tilted", 2, 2000),
    (256, 256, 64, 32, "tilted", 0, 2000),
])
def test_full_size_runs_match_oracle(hs, orc, W, H, N, S, kind, tour, G):
    kinds = {"steady": 0, "tilted": 1, "hybrid": 2}
    cfg = hs.Config(W, H, N, S, kind, tournament_size=tour, seed=1)
    run = hs.Run(cfg)
    run.step(G)
    run.sync()
    o = orc.Run(W, H, N, S, kinds[kind], tournament=tour, seed=1, threads=THREADS)
    oracle_steps(o, G, f"{W}x{H}x{N} {kind}-{S} tournament {tour}")
    for name, x, y in zip(("trait", "counter", "surface"), run.agents(), o.agents()):
        assert np.array_equal(x, y), name
    assert np.array_equal(run.layout(), o.layout())
    for x, y in zip(run.outbox(), o.outbox()):
        assert np.array_equal(x, y)
    o.close()
    # the benchmark's query on the evolved population: a 4,096-agent sample,
    # every one of its 16,777,216 ordered pairs, and the reconstructed tree
    _, cnt, srf = run.sample(4096)
    cnt_h, srf_h = hs.as_u32(cnt), hs.as_u32(srf)
    lb, ub = hs.mrca_bounds(kind, S, cnt, srf)
    olb, oub = orc.mrca_allpairs(kinds[kind], S, cnt_h, srf_h)
    assert np.array_equal(hs.as_u32(lb), olb) and np.array_equal(hs.as_u32(ub), oub)
    got = hs.phylo_metrics(kind, S, cnt, srf)
    sbl, pairs, root, internal, ed = orc.phylo_metrics(kinds[kind], S, cnt_h, srf_h)
    assert (got["sum_branch_length"], got["pair_sum"], got["root_time"],
            got["internal_nodes"]) == (sbl, pairs, root, internal)
    # the benchmark's own route: the run-bound query takes the run's layout
    rlb, rub = run.mrca_bounds(cnt, srf)
    assert np.array_equal(hs.as_u32(rlb), olb) and np.array_equal(hs.as_u32(rub), oub)
    rt = run.phylo_tree(cnt, srf, tree=False)
    assert (rt["sum_branch_length"], rt["pair_sum"], rt["root_time"],
            rt["internal_nodes"]) == (sbl, pairs, root, internal)


def test_full_size_float_trial_matches_oracle(hs, orc):
    """The adaptation-enabled treatment (deleterious and beneficial
    mutations both occur)."""
    G, ben = 100, 12884901
    cfg = hs.Config(750, 750, 32, 64, "tilted", tournament_size=5, seed=1,
                    fitness_model="float", del_threshold=1417339207, ben_threshold=ben)
    run = hs.Run(cfg)
    run.step(G)
    run.sync()
    o = orc.Run(750, 750, 32, 64, 1, tournament=5, seed=1, fitness_model=orc.FLOAT_FITNESS,
                del_thr=1417339207, ben_thr=ben, threads=THREADS)
    oracle_steps(o, G, f"float trial, beneficial threshold {ben}")
    for name, x, y in zip(("fitness", "counter", "surface"), run.agents(), o.agents()):
        assert np.array_equal(x, y), name
    assert np.array_equal(run.layout(), o.layout())
    for x, y in zip(run.outbox(), o.outbox()):
        assert np.array_equal(x, y)
    o.close()


def test_full_size_asynchronous_ticks_match_oracle(hs, orc):
    G = 200
    act = int(0.9 * 2**32)
    cfg = hs.Config(512, 1024, 32, 64, "hybrid", tournament_size=2, seed=1, async_activity=act)
    run = hs.Run(cfg, max_gens_per_launch=G)
    run.step(G)
    run.sync()
    o = orc.Run(512, 1024, 32, 64, 2, tournament=2, seed=1, activity=act, threads=THREADS)
    oracle_steps(o, G, "asynchronous ticks")
    for name, x, y in zip(("trait", "counter", "surface"), run.agents(), o.agents()):
        assert np.array_equal(x, y), name
    assert np.array_equal(run.layout(), o.layout())
    for x, y in zip(run.outbox(), o.outbox()):
        assert np.array_equal(x, y)
    o.close()
