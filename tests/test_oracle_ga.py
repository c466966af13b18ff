"""Pins of the oracle's GA step.

The paper prints no run to compare with, so the step itself is "parity
unpinned" against the paper.  These tests pin it by special cases,
invariants and the recorded pedigree (Methods, Asynchronous Island-model
Genetic Algorithm and Genome Model):

* every child is a copy of one parent from its island's population after
  immigration, with the counter incremented, the trait changed by at most
  the mutation range, and the surface changed only at this generation's
  site, where it holds the differentia bit drawn at birth;
* parents come from the island or from a neighbour whose emigrant was
  addressed to it;
* a tournament among equal traits keeps the first draw, so it reduces to
  neutral selection;
* without migration, island histories do not depend on the torus shape;
* selection raises the mean trait; neutral drift keeps it near zero;
* the differentia at each retained site equals the bit drawn at the birth
  of the generation-(t+1) ancestor.
"""
import numpy as np
import pytest

KIND = {"steady": 0, "tilted": 1, "hybrid": 2}


def neighbour(W, H, i, d):
    x, y = i % W, i // W
    if d == 0:
        y = (y - 1) % H
    elif d == 1:
        y = (y + 1) % H
    elif d == 2:
        x = (x - 1) % W
    else:
        x = (x + 1) % W
    return y * W + x


def test_counters_and_layout(orc):
    r = orc.Run(4, 4, 8, 32, KIND["steady"], seed=3)
    for g in (1, 5, 40):
        r.step(g - r.generation)
        t, c, s = r.agents()
        assert np.all(c == g)
        assert np.array_equal(r.layout(), orc.layout(0, 32, g))


def test_no_mutation_keeps_traits_zero(orc):
    r = orc.Run(4, 2, 16, 64, KIND["hybrid"], mut_thr=0, seed=9)
    r.step(100)
    t, c, s = r.agents()
    assert np.all(t == 0)
    assert np.any(s != 0)


def test_tournament_of_ties_is_neutral(orc):
    """With no mutation all traits stay 0: every tournament is a tie and
    keeps the first draw, which is the neutral parent."""
    a = orc.Run(3, 2, 8, 32, 1, tournament=2, mut_thr=0, seed=5, pedigree_gens=30)
    b = orc.Run(3, 2, 8, 32, 1, tournament=0, mut_thr=0, seed=5, pedigree_gens=30)
    a.step(30)
    b.step(30)
    for g in range(1, 31):
        assert np.array_equal(a.pedigree(g)[0], b.pedigree(g)[0])
    for x, y in zip(a.agents(), b.agents()):
        assert np.array_equal(x, y)


def test_islands_independent_without_migration(orc):
    """Each island's draws are keyed by its own index only."""
    runs = [orc.Run(W, H, 8, 32, 1, migrants=0, seed=11) for W, H in
            ((2, 2), (2, 3), (4, 1))]
    for r in runs:
        r.step(60)
    states = [r.agents() for r in runs]
    n = 4 * 8
    for st in states[1:]:
        for x, y in zip(states[0], st):
            assert np.array_equal(x[:n], y[:n])
    assert all(r.outbox() is None for r in runs)


@pytest.mark.parametrize("W,H", [(3, 4), (1, 1), (2, 1), (1, 3)])
def test_births_follow_the_step_definition(orc, W, H):
    N, S = 8, 64
    G = 40
    r = orc.Run(W, H, N, S, KIND["hybrid"], seed=7, pedigree_gens=G)
    prev = r.agents()
    prev_L = r.layout()
    prev_ob = r.outbox()
    total_immigrants = 0
    for g in range(G):
        r.step(1)
        t, c, s = r.agents()
        L = r.layout()
        changed = np.nonzero(L != prev_L)[0]
        assert len(changed) == 1 and L[changed[0]] == g
        site = int(changed[0])
        parent, bit = r.pedigree(g + 1)
        pt, pc, ps = prev
        for a in range(r.A):
            p = int(parent[a])
            i = a // N
            allowed_islands = {i}
            if prev_ob is not None:
                d_, _, _, _, src = prev_ob
                for d in range(4):
                    nb = neighbour(W, H, i, d)
                    if d_[nb] == (d ^ 1):
                        allowed_islands.add(int(src[nb]) // N)
            assert p // N in allowed_islands
            assert c[a] == pc[p] + 1
            delta = ((int(t[a]) - int(pt[p]) + 2**31) % 2**32) - 2**31
            assert -8 <= delta <= 8
            want = ps[p].copy()
            w, b = divmod(site, 32)
            want[w] = (int(want[w]) & ~(1 << b)) | (int(bit[a]) << b)
            assert np.array_equal(s[a], want)
        if prev_ob is not None:
            d_ = prev_ob[0]
            total_immigrants += sum(
                1 for i in range(r.I) for d in range(4)
                if d_[neighbour(W, H, i, d)] == (d ^ 1))
        ob = r.outbox()
        assert ob is not None
        d_, ot, oc, os_, src = ob
        # the emigrant is a copy of a member of the island's new population
        for i in range(r.I):
            e = int(src[i])
            assert e // N == i
            assert ot[i] == t[e] and oc[i] == c[e]
            assert np.array_equal(os_[i], s[e])
            assert d_[i] < 4
        prev, prev_L, prev_ob = (t, c, s), L, ob
    # one emigrant per island per generation arrives somewhere
    assert total_immigrants == (G - 1) * r.I


def test_immigrants_become_parents(orc):
    """Immigrants overwrite members before the births (migration first), so
    some children descend from a neighbour island's emigrant: under neutral
    selection each birth picks any member of the island after immigration
    with probability 1/N, so the children with a parent from another island
    number about the immigrants written, about one per island per
    generation (each emigrant goes to one of the four neighbours)."""
    W, H, N, G = 4, 4, 8, 100
    r = orc.Run(W, H, N, 32, KIND["tilted"], tournament=0, seed=13, pedigree_gens=G)
    r.step(G)
    foreign = 0
    for g in range(2, G + 1):          # generation 0 has no outbox to read
        parent, _ = r.pedigree(g)
        foreign += int(np.sum(parent.astype(np.int64) // N != np.arange(r.A) // N))
    expect = r.I * (G - 1)
    assert 0.8 * expect < foreign < 1.15 * expect, (foreign, expect)


def test_emigrant_directions_are_uniform(orc):
    """Each generation's emigrant goes to a uniformly chosen one of the four
    cardinal neighbours."""
    r = orc.Run(4, 4, 8, 32, KIND["steady"], seed=17)
    counts = np.zeros(4)
    for _ in range(100):
        r.step(1)
        d = r.outbox()[0]
        counts += np.bincount(d.astype(np.int64), minlength=4)[:4]
    expect = counts.sum() / 4
    chi2 = float(np.sum((counts - expect) ** 2 / expect))
    assert chi2 < 16.27, counts     # 3 degrees of freedom, p = 0.001


def test_mutation_statistics(orc):
    r = orc.Run(8, 8, 32, 32, 0, tournament=0, seed=21, pedigree_gens=100)
    prev_t = r.agents()[0]
    changes = []
    for g in range(100):
        r.step(1)
        t = r.agents()[0]
        parent, _ = r.pedigree(g + 1)
        changes.append((t - prev_t[parent]).astype(np.int32))
        prev_t = t
    d = np.concatenate(changes)
    births = d.size
    nz = d[d != 0]
    # mutation with p = 0.01, uniform on 17 values [-8, 8], so p * 16/17 change
    expect = births * 0.01 * 16 / 17
    assert abs(nz.size - expect) < 5 * np.sqrt(expect)
    assert nz.min() >= -8 and nz.max() <= 8
    assert set(np.unique(nz).tolist()) == set(range(-8, 9)) - {0}


def test_selection_raises_mean_trait(orc):
    sel = orc.Run(8, 8, 32, 32, 0, tournament=2, seed=1)
    neu = orc.Run(8, 8, 32, 32, 0, tournament=0, seed=1)
    sel.step(600)
    neu.step(600)
    ms = sel.agents()[0].astype(np.int32).mean()
    mn = neu.agents()[0].astype(np.int32).mean()
    assert ms > 20.0          # beneficial mutations sweep under selection
    assert abs(mn) < 15.0     # neutral drift: a martingale around 0


def test_determinism_and_seed_sensitivity(orc):
    a = orc.Run(4, 4, 16, 32, 1, seed=2)
    b = orc.Run(4, 4, 16, 32, 1, seed=2)
    c = orc.Run(4, 4, 16, 32, 1, seed=3)
    for r in (a, b, c):
        r.step(50)
    for x, y in zip(a.agents(), b.agents()):
        assert np.array_equal(x, y)
    assert not np.array_equal(a.agents()[2], c.agents()[2])


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_pedigree_consistency(orc, kind):
    """The bit at a retained site holding item t is the differentia drawn at
    the birth of the agent's generation-(t+1) ancestor."""
    W, H, N, S, G = 2, 2, 4, 32, 150
    r = orc.Run(W, H, N, S, kind, seed=4, pedigree_gens=G)
    r.step(G)
    ped = [None] + [r.pedigree(g) for g in range(1, G + 1)]
    t, c, s = r.agents()
    L = r.layout()
    for a in range(r.A):
        anc = {G: a}
        for g in range(G, 0, -1):
            anc[g - 1] = int(ped[g][0][anc[g]])
        for k in range(S):
            item = int(L[k])
            want = int(ped[item + 1][1][anc[item + 1]])
            got = (int(s[a][k // 32]) >> (k % 32)) & 1
            assert got == want, (a, k, item)


def test_invalid_configs_rejected(orc):
    with pytest.raises(ValueError):
        orc.Run(0, 4, 8, 32, 0)
    with pytest.raises(ValueError):
        orc.Run(4, 4, 65, 32, 0)
    with pytest.raises(ValueError):
        orc.Run(4, 4, 8, 48, 0)
    with pytest.raises(ValueError):
        orc.Run(4, 4, 8, 32, 0, mut_lo=3, mut_hi=2)
    with pytest.raises(ValueError):
        orc.Run(4, 4, 8, 32, 3)


@pytest.mark.parametrize("kw", [dict(kind=2, S=64, tournament=2),
                                dict(kind=1, S=32, tournament=0, N=17),
                                dict(kind=0, S=8, bits=8, interval=3, tournament=2)])
def test_island_threaded_oracle_equals_serial(orc, kw):
    """The island-parallel births (one barrier per generation) give the
    serial oracle's result word for word, pedigree included."""
    kw = dict(kw)
    N = kw.pop("N", 8)
    kind, S = kw.pop("kind"), kw.pop("S")
    G = 60
    runs = [orc.Run(5, 3, N, S, kind, seed=29, pedigree_gens=G, threads=t, **kw)
            for t in (0, 4, 15)]
    for r in runs:
        r.step(G)
    want = runs[0].agents()
    for r in runs[1:]:
        for x, y in zip(want, r.agents()):
            assert np.array_equal(x, y)
        assert np.array_equal(runs[0].layout(), r.layout())
        for x, y in zip(runs[0].outbox(), r.outbox()):
            assert np.array_equal(x, y)
        for g in (1, G // 2, G):
            for x, y in zip(runs[0].pedigree(g), r.pedigree(g)):
                assert np.array_equal(x, y)
