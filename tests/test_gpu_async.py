"""GPU parity of asynchronous runs against the oracle (zero tolerance):
islands active per tick with a given probability, per-agent counters,
deposits at the site each parent's own counter selects (constant-time
lookups in the rule's tables), idle islands posting nothing; all birth models and annotation
schemes, migration on and off, every tick of a small run, launch shapes,
the synchronous reduction, MRCA bounds of drifting counters, and the
limits."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

KINDS = ("steady", "tilted", "hybrid")
P = lambda p: int(p * 2**32)          # noqa: E731


@pytest.fixture(scope="module")
def hs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_10861_amd as hs
    hs.load_library()
    return hs


def acfg(hs, W, H, N, kind, S, activity, bits=1, interval=1, seed=3, **kw):
    return hs.Config(W, H, N, S, KINDS[kind], seed=seed, differentia_bits=bits,
                     ingest_interval=interval, async_activity=activity, **kw)


def oracle_for(orc, c):
    model = {"int": 0, "float": 1, "tag": 2}[c.fitness_model]
    return orc.Run(c.grid_w, c.grid_h, c.pop_per_island, c.surface_sites, c.kind,
                   tournament=c.tournament_size, mut_thr=c.mut_threshold, mut_lo=c.mut_lo,
                   mut_hi=c.mut_hi, migrants=c.migrants_per_island, seed=c.seed,
                   fitness_model=model, del_thr=c.del_threshold, ben_thr=c.ben_threshold,
                   del_sigma=c.del_sigma, ben_sigma=c.ben_sigma, bits=c.differentia_bits,
                   interval=c.ingest_interval, activity=c.async_activity)


def same_state(run, o):
    for x, y in zip(run.agents(), o.agents()):
        assert np.array_equal(x, y)
    assert np.array_equal(run.layout(), o.layout())
    ob, oo = run.outbox(), o.outbox()
    assert (ob is None) == (oo is None)
    if ob is not None:
        for x, y in zip(ob, oo):
            assert np.array_equal(x, y)


MODELS = {"int": dict(tournament_size=2),
          "float": dict(fitness_model="float", tournament_size=5, del_threshold=1417339207,
                        ben_threshold=128849010),
          "tag": dict(fitness_model="tag", tournament_size=0)}


@pytest.mark.parametrize("activity", [0.3, 0.7, 0.97])
@pytest.mark.parametrize("model", ["int", "float", "tag"])
@pytest.mark.parametrize("scheme", [(1, 32, 1, 1), (2, 64, 1, 3), (0, 8, 8, 1)])
@pytest.mark.parametrize("migrants", [1, 0])
def test_runs_match_oracle(hs, orc, activity, model, scheme, migrants):
    kind, S, bits, interval = scheme
    c = acfg(hs, 7, 5, 16, kind, S, P(activity), bits, interval, seed=int(activity * 100),
             migrants_per_island=migrants, **MODELS[model])
    run = hs.Run(c, max_gens_per_launch=400)
    run.step(400)
    o = oracle_for(orc, c)
    o.step(400)
    same_state(run, o)


def test_every_tick(hs, orc):
    c = acfg(hs, 6, 6, 32, 2, 64, P(0.6), interval=2, seed=9)
    run = hs.Run(c, max_gens_per_launch=256)
    o = oracle_for(orc, c)
    for k in range(150):
        run.step(1)
        o.step(1)
        for x, y in zip(run.agents(), o.agents()):
            assert np.array_equal(x, y), k
    same_state(run, o)


@pytest.mark.parametrize("block,apt", [(64, 1), (128, 2), (256, 4), (1024, 2)])
def test_launch_shapes(hs, orc, block, apt):
    c = acfg(hs, 9, 7, 32, 1, 32, P(0.8), seed=4)
    run = hs.Run(c, max_gens_per_launch=300)
    run.set_launch_shape(block, apt)
    run.step(300)
    o = oracle_for(orc, c)
    o.step(300)
    same_state(run, o)


def test_split_steps(hs, orc):
    """Ticks enqueued in uneven pieces."""
    c = acfg(hs, 5, 5, 16, 0, 8, P(0.5), bits=8, interval=3, seed=6)
    run = hs.Run(c, max_gens_per_launch=200)
    for n in (1, 5, 2, 30, 7, 55):
        run.step(n)
    o = oracle_for(orc, c)
    o.step(100)
    same_state(run, o)


def test_all_active_equals_synchronous(hs, orc):
    c = acfg(hs, 8, 8, 32, 2, 64, 0xFFFFFFFF, seed=12)
    for k in range(200):
        for i in range(64):
            assert orc.philox(0, i, k, orc.ACTIVITY, 12)[0] < 0xFFFFFFFF
    a = hs.Run(c, max_gens_per_launch=200)
    a.step(200)
    sync = hs.Config(8, 8, 32, 64, "hybrid", seed=12)
    b = hs.Run(sync)
    b.step(200)
    for x, y in zip(a.agents(), b.agents()):
        assert np.array_equal(x, y)
    assert np.array_equal(a.layout(), b.layout())


def test_bounds_of_drifting_counters(hs, orc):
    c = acfg(hs, 16, 16, 32, 2, 64, P(0.75), seed=21)
    run = hs.Run(c, max_gens_per_launch=1000)
    run.step(1000)
    _, cnt, srf = run.sample(600)
    cnt_h, srf_h = hs.as_u32(cnt), hs.as_u32(srf)
    assert len(np.unique(cnt_h)) > 10                 # islands drifted apart
    lb, ub = hs.mrca_bounds("hybrid", 64, cnt, srf)
    olb, oub = orc.mrca_allpairs(2, 64, cnt_h, srf_h)
    assert np.array_equal(hs.as_u32(lb), olb) and np.array_equal(hs.as_u32(ub), oub)
    assert hs.phylo_metrics("hybrid", 64, cnt, srf)["status"] == 1


@pytest.mark.parametrize("kind,S,bits,interval,ticks", [(2, 64, 1, 1, 3000), (1, 32, 1, 1, 5000),
                                                         (0, 8, 8, 3, 4000)])
def test_no_tick_limit(hs, orc, kind, S, bits, interval, ticks):
    """Births look sites up in the rule's constant-time tables, so a run is
    not bounded by its launch batch: a run created with 64 generations per
    launch steps thousands of ticks, in uneven pieces, equal to the oracle
    (whose lookups replay the placements)."""
    c = acfg(hs, 6, 5, 16, kind, S, P(0.85), bits, interval, seed=31)
    run = hs.Run(c, max_gens_per_launch=64)
    done = 0
    for piece in (1, 63, 700, ticks - 764):
        run.step(piece)
        done += piece
    assert done == ticks
    o = oracle_for(orc, c)
    o.step(ticks)
    same_state(run, o)
    counters = run.agents()[1]
    assert counters.max() > 64 and len(np.unique(counters)) > 5


def test_limits(hs):
    c = acfg(hs, 4, 4, 8, 1, 32, P(0.5))
    pool = hs.Pool(8 << 20, max_runs=2, max_gens_per_launch=16)
    with pytest.raises(hs.HsgaError):
        pool.admit(c, 10)
    pool.close()
    # the horizon still binds: hybrid-8 byte surfaces place 2 (2^4 - 2) + 2 items
    h = acfg(hs, 2, 2, 4, 2, 8, P(0.5), bits=8)
    run = hs.Run(h)
    with pytest.raises(hs.HsgaError) as e:
        run.step(2 * (2**4 - 2) + 2 + 2)
    assert e.value.status == hs.GA_EHORIZON
