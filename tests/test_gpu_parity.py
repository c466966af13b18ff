"""GPU parity: the HIP path (through the C ABI) against the oracle, bit for
bit on every agent word, outbox entry and layout site.  Everything here is
integer work, so the tolerance is zero.
"""
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


def make_pair(hs, orc, W, H, N, S, kind, tournament=2, migrants=1, seed=1,
              mut_thr=42949672, mut_lo=-8, mut_hi=8, gens_per_launch=0):
    cfg = hs.Config(W, H, N, S, kind, tournament, mut_thr, mut_lo, mut_hi, migrants, seed)
    g = hs.Run(cfg, max_gens_per_launch=gens_per_launch)
    o = orc.Run(W, H, N, S, KIND[kind], tournament, mut_thr, mut_lo, mut_hi, migrants, seed)
    return g, o


def assert_same_state(g, o, where=""):
    gt, gc, gs = g.agents()
    ot, oc, os_ = o.agents()
    assert np.array_equal(gt, ot), f"trait differs {where}: first at {np.argmax(gt != ot)}"
    assert np.array_equal(gc, oc), f"counter differs {where}"
    assert np.array_equal(gs, os_), f"surface differs {where}: first agent {np.argmax(np.any(gs != os_, axis=1))}"
    assert np.array_equal(g.layout(), o.layout()), f"layout differs {where}"
    gob, oob = g.outbox(), o.outbox()
    assert (gob is None) == (oob is None), where
    if gob is not None:
        for x, y, name in zip(gob, oob[:4], ("dir", "trait", "counter", "surface")):
            assert np.array_equal(x, y), f"outbox {name} differs {where}"


def test_c1_every_generation(hs, orc):
    """The CPU-scale workload, compared after every generation."""
    g, o = make_pair(hs, orc, 8, 8, 32, 32, "steady", seed=1, gens_per_launch=64)
    assert_same_state(g, o, "at founders")
    for gen in range(1, 1001):
        g.step(1)
        o.step(1)
        if gen <= 100 or gen % 10 == 0:
            assert_same_state(g, o, f"at generation {gen}")
    assert_same_state(g, o, "at generation 1000")


@pytest.mark.parametrize("kind", ["steady", "tilted", "hybrid"])
@pytest.mark.parametrize("S", [32, 64])
@pytest.mark.parametrize("tournament", [2, 0])
def test_kinds_sizes_treatments(hs, orc, kind, S, tournament):
    g, o = make_pair(hs, orc, 6, 5, 16, S, kind, tournament=tournament, seed=7)
    for chunk in (1, 2, 37, 160):
        g.step(chunk)
        o.step(chunk)
        assert_same_state(g, o, f"{kind} S={S} T={g.generation}")


@pytest.mark.parametrize("W,H,N", [(1, 1, 8), (2, 1, 4), (1, 3, 64), (5, 3, 3), (7, 9, 48),
                                   (33, 2, 1), (3, 35, 2), (4, 4, 64), (13, 11, 32), (9, 7, 17)])
def test_torus_shapes_and_population_sizes(hs, orc, W, H, N):
    """Degenerate tori (1x1, 2x1, 1x3), populations that do not divide the
    wavefront (3, 17, 48), and island counts that leave ragged tails."""
    g, o = make_pair(hs, orc, W, H, N, 64, "hybrid", seed=3)
    g.step(90)
    o.step(90)
    assert_same_state(g, o, f"{W}x{H}x{N}")


def test_migration_off(hs, orc):
    g, o = make_pair(hs, orc, 8, 4, 32, 32, "tilted", migrants=0, seed=5)
    g.step(200)
    o.step(200)
    assert_same_state(g, o)
    assert g.outbox() is None


def test_no_mutation_and_wide_mutation(hs, orc):
    for thr, lo, hi in ((0, -8, 8), (2**32 - 1, -1000, 1000), (2**31, 0, 0)):
        g, o = make_pair(hs, orc, 4, 4, 32, 32, "steady", seed=11, mut_thr=thr, mut_lo=lo,
                         mut_hi=hi)
        g.step(50)
        o.step(50)
        assert_same_state(g, o, f"thr={thr} [{lo},{hi}]")


@pytest.mark.parametrize("block,apt", [(64, 1), (128, 2), (256, 4), (1024, 2), (192, 2),
                                       (1024, 1), (512, 4), (64, 4)])
def test_launch_shape_invariance(hs, orc, block, apt):
    g, o = make_pair(hs, orc, 16, 12, 32, 64, "hybrid", seed=13)
    g.set_launch_shape(block, apt)
    g.step(75)
    o.step(75)
    assert_same_state(g, o, f"block={block} apt={apt}")


def test_launch_shape_rejects_bad_shapes(hs):
    g = hs.Run(hs.Config(4, 4, 48, 32, "steady"))
    for block, apt in ((100, 4), (2048, 4), (256, 3), (256, 32)):
        with pytest.raises(hs.HsgaError):
            g.set_launch_shape(block, apt)
    g2 = hs.Run(hs.Config(4, 4, 17, 32, "steady"))
    with pytest.raises(hs.HsgaError):
        g2.set_launch_shape(256, 2)       # 2 does not divide 17


def test_chunked_site_schedule(hs, orc):
    """Schedules split across launches (3 generations per launch)."""
    g, o = make_pair(hs, orc, 4, 4, 16, 32, "tilted", seed=17, gens_per_launch=3)
    g.step(100)
    o.step(100)
    assert_same_state(g, o)


@pytest.mark.parametrize("tournament", [2, 0])
def test_treatment_pair_scaled_down_full_length(hs, orc, tournament):
    """The treatment-pair workload on a 12x12 torus, its full 20,000
    generations (the 256x256 version is checked by properties below)."""
    g, o = make_pair(hs, orc, 12, 12, 64, 32, "tilted", tournament=tournament, seed=1)
    g.step(20000)
    o.step(20000)
    assert_same_state(g, o)


def test_paper_scale_past_the_fill_phase(hs, orc):
    """The 16.8 M-agent hybrid-64 workload in the launch configuration the
    benchmark times, every word after 100 generations: both 32-site halves
    fill by generation 63, so generations 64..99 overwrite evicted sites
    on the full torus.  Then the benchmark's query route (a 4,096-agent
    stratified sample, all 16.8 M ordered pairs of MRCA bounds from the
    run's own layout) against the oracle, pair for pair.  The oracle runs
    its island-parallel births on 16 host threads."""
    import os
    cfg = hs.Config(512, 1024, 32, 64, "hybrid", seed=1)
    g = hs.Run(cfg, max_gens_per_launch=10000)
    o = orc.Run(512, 1024, 32, 64, KIND["hybrid"], seed=1,
                threads=min(16, os.cpu_count() or 1))
    g.step(100)
    o.step(100)
    assert_same_state(g, o, "at generation 100")
    layout = o.layout()
    assert np.all(layout != orc.EMPTY) and layout.max() == 99
    _, cnt, srf = g.sample(4096)
    lb, ub = g.mrca_bounds(cnt, srf)
    idx = orc.sample(1, cfg.agents, 4096, 100)
    _, oc, os_ = o.agents()
    olb, oub = orc.mrca_allpairs(KIND["hybrid"], 64, oc[idx], os_[idx])
    assert np.array_equal(hs.as_u32(lb), olb)
    assert np.array_equal(hs.as_u32(ub), oub)


def test_horizon_is_refused(hs):
    cfg = hs.Config(2, 2, 4, 32, "hybrid", seed=1)
    g = hs.Run(cfg)
    with pytest.raises(hs.HsgaError) as e:
        g.step(2 * (2**16 - 2) + 3 + 1)
    assert e.value.status == -3
    assert g.generation == 0


def test_invalid_configs(hs):
    for bad in (dict(grid_w=0, grid_h=4), dict(grid_w=4, grid_h=4, pop_per_island=65),
                dict(grid_w=4, grid_h=4, surface_sites=48),
                dict(grid_w=4, grid_h=4, tournament_size=3),
                dict(grid_w=4, grid_h=4, mut_lo=2, mut_hi=1)):
        with pytest.raises(hs.HsgaError) as e:
            hs.Run(hs.Config(**bad))
        assert e.value.status == -1


def test_determinism_across_runs(hs):
    cfg = hs.Config(16, 16, 32, 64, "hybrid", seed=99)
    a = hs.Run(cfg)
    b = hs.Run(cfg)
    b.set_launch_shape(512, 2)
    a.step(300)
    b.step(300)
    for x, y in zip(a.agents(), b.agents()):
        assert np.array_equal(x, y)
    # another seed: other draws, so other traits and annotations
    c = hs.Run(hs.Config(16, 16, 32, 64, "hybrid", seed=100))
    c.step(300)
    ta, _, sa = a.agents()
    tc, _, sc = c.agents()
    assert not np.array_equal(ta, tc) and not np.array_equal(sa, sc)


@pytest.mark.parametrize("kind", ["steady", "tilted", "hybrid"])
@pytest.mark.parametrize("S", [32, 64])
def test_site_schedule_past_2_16(hs, orc, kind, S):
    """The device schedule (leave-time form of the retention target) equals
    the oracle's placement over 70,000 generations, in uneven chunks."""
    g = hs.Run(hs.Config(1, 1, 2, S, kind, seed=3), max_gens_per_launch=9000)
    done = 0
    for chunk in (1, 31, 33, 5000, 9000, 30000, 25935):
        g.step(chunk)
        done += chunk
        assert np.array_equal(g.layout(), orc.layout(KIND[kind], S, done)), done
    assert done == 70000


@pytest.mark.parametrize("nbytes", [16, 4096 + 16, (1 << 20) + 48])
def test_probe_copy_is_exact(hs, nbytes):
    """The instrumentation copy moves exactly the requested 16-byte multiple
    (ragged last workgroup included) and nothing beyond it."""
    import torch
    rng = np.random.default_rng(nbytes)
    src_h = rng.integers(0, 256, size=nbytes + 64, dtype=np.uint8)
    src = torch.from_numpy(src_h).cuda()
    dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")
    moved = hs.probe_copy(src[:nbytes], dst)
    torch.cuda.synchronize()
    out = dst.cpu().numpy()
    assert moved == nbytes
    assert np.array_equal(out[:nbytes], src_h[:nbytes])
    assert not out[nbytes:].any()
