"""The resident form of small synchronous runs (one workgroup takes the
whole torus through a launch batch's generations): bit for bit against the
oracle and against the same run stepped one launch per generation, over
the birth models, surfaces, schemes, agents per thread (N divisible by 4,
by 2 only, by neither), a single island, the largest run that steps
resident, launch batches that split a step, and single generations."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

KIND = {"steady": 0, "tilted": 1, "hybrid": 2}


@pytest.fixture(scope="module")
def hs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_10861_amd as hs
    hs.load_library()
    return hs


def oracle_for(orc, c):
    model = {"int": 0, "float": 1, "tag": 2}[c.fitness_model]
    return orc.Run(c.grid_w, c.grid_h, c.pop_per_island, c.surface_sites,
                   KIND[c.surface_kind], tournament=c.tournament_size,
                   mut_thr=c.mut_threshold, mut_lo=c.mut_lo, mut_hi=c.mut_hi,
                   migrants=c.migrants_per_island, seed=c.seed, fitness_model=model,
                   del_thr=c.del_threshold, ben_thr=c.ben_threshold, del_sigma=c.del_sigma,
                   ben_sigma=c.ben_sigma, bits=c.differentia_bits, interval=c.ingest_interval)


def same_state(a, b, where=""):
    for x, y, name in zip(a.agents(), b.agents(), ("trait", "counter", "surface")):
        assert np.array_equal(x, y), f"{name} differs {where}"
    assert np.array_equal(a.layout(), b.layout()), f"layout differs {where}"
    oa, ob = a.outbox(), b.outbox()
    assert (oa is None) == (ob is None), where
    if oa is not None:
        for x, y in zip(oa, ob):
            assert np.array_equal(x, y), f"outbox differs {where}"


FLOAT = dict(fitness_model="float", tournament_size=5, del_threshold=1417339207,
             ben_threshold=128849010)

CASES = [
    # W, H, N, S, kind, extra config
    (8, 8, 32, 32, "steady", dict(tournament_size=2)),              # the CPU-scale workload
    (9, 7, 32, 64, "hybrid", dict(tournament_size=2)),
    (4, 4, 48, 32, "tilted", dict(tournament_size=0)),
    (3, 5, 6, 64, "hybrid", dict(tournament_size=2)),               # 2 agents per thread
    (5, 5, 7, 32, "steady", dict(tournament_size=2)),               # 1 agent per thread
    (1, 1, 32, 64, "hybrid", dict(tournament_size=2)),              # one island
    (16, 16, 16, 32, "tilted", dict(tournament_size=2)),            # 4,096 agents
    (8, 8, 32, 64, "tilted", FLOAT),
    (6, 6, 16, 64, "hybrid", dict(FLOAT, ben_threshold=0)),
    (8, 4, 32, 64, "tilted", dict(fitness_model="tag", tournament_size=0)),
    (8, 8, 32, 8, "hybrid", dict(differentia_bits=8, ingest_interval=2, tournament_size=2)),
    (5, 6, 32, 32, "steady", dict(ingest_interval=3, tournament_size=0)),
    (7, 7, 32, 32, "tilted", dict(migrants_per_island=0, tournament_size=2)),
]


@pytest.mark.parametrize("W,H,N,S,kind,extra", CASES)
def test_resident_matches_oracle_and_plain_launches(hs, orc, W, H, N, S, kind, extra):
    c = hs.Config(W, H, N, S, kind, seed=5, **extra)
    res = hs.Run(c, max_gens_per_launch=64)
    plain = hs.Run(c, max_gens_per_launch=64)
    plain.set_resident(False)
    assert res.resident_threads > 0 and plain.resident_threads == 0
    o = oracle_for(orc, c)
    # steps that span launch batches (64 generations each), and single ones,
    # up to the scheme's horizon
    left = min(200, orc.horizon_gen(KIND[kind], S, c.ingest_interval) + 1)
    for n in (1, 7, 64, 78, 1, 49):
        n = min(n, left)
        if n == 0:
            break
        left -= n
        res.step(n)
        plain.step(n)
        o.step(n)
        same_state(res, plain, f"after a step of {n} (resident vs plain launches)")
        same_state(res, o, f"after a step of {n} (resident vs oracle)")


def test_resident_every_generation(hs, orc):
    """The CPU-scale workload one generation per call."""
    c = hs.Config(8, 8, 32, 32, "steady", tournament_size=2, seed=1)
    res = hs.Run(c, max_gens_per_launch=64)
    assert res.resident_threads == 512
    o = oracle_for(orc, c)
    for gen in range(1, 121):
        res.step(1)
        o.step(1)
        same_state(res, o, f"at generation {gen}")


def test_resident_form_applies_only_where_it_fits(hs):
    assert hs.Run(hs.Config(8, 8, 32, 32, "steady")).resident_threads == 512
    assert hs.Run(hs.Config(16, 16, 16, 32, "steady")).resident_threads == 1024
    r = hs.Run(hs.Config(5, 5, 7, 32, "steady"))          # 1 agent per thread: 175 threads
    assert r.resident_threads == 192
    assert hs.Run(hs.Config(16, 16, 32, 32, "steady")).resident_threads == 0     # 8,192 agents
    act = int(0.9 * 2**32)
    assert hs.Run(hs.Config(8, 8, 32, 32, "steady", async_activity=act)).resident_threads == 0
    r = hs.Run(hs.Config(8, 8, 32, 32, "steady"))
    r.set_resident(False)
    assert r.resident_threads == 0
    r.set_resident(True)
    assert r.resident_threads == 512


def test_resident_kernel_time_counts_generations(hs):
    r = hs.Run(hs.Config(8, 8, 32, 32, "steady", seed=2), max_gens_per_launch=64)
    r.set_kernel_timing(True)
    r.step(150)
    ms, n = r.kernel_time()
    assert n == 150 and ms > 0
