"""Pins of the oracle's annotation schemes and founder tags.

* Byte differentiae (Distributed Phylogenetic Tracking: differentiae of a
  bit or a byte; wider ones collide less) and coarsened ingest (Results,
  Surface Algorithm Benchmark: update annotations only every n-th
  generation): the MRCA bounds against the true pedigree, the retained
  values against the values drawn at the ancestors' births, generations
  between ingests leaving annotations untouched, the horizon in
  generations, and a hand-worked many-way reconstruction.
* Founder tags (Genome Model; Results, Clade Reconstruction Trial): random
  16-bit identifiers inherited without mutation under neutral selection.
"""
import numpy as np
import pytest

# (kind, S sites, bits per differentia, ingest interval)
SCHEMES = [(0, 8, 8, 1), (1, 8, 8, 2), (2, 8, 8, 1), (0, 4, 8, 5), (1, 32, 1, 3),
           (0, 64, 1, 4), (2, 32, 1, 2), (2, 64, 1, 7)]


def value(s, k, bits):
    per = 32 // bits
    return (int(s[k // per]) >> ((k % per) * bits)) & ((1 << bits) - 1)


def lineage(ped, G, a):
    anc = {G: a}
    for g in range(G, 0, -1):
        anc[g - 1] = int(ped[g][0][anc[g]])
    return anc


def run_with_pedigree(orc, kind, S, bits, interval, G, seed=1, **kw):
    r = orc.Run(2, 2, 4, S, kind, seed=seed, pedigree_gens=G, bits=bits, interval=interval,
                **kw)
    r.step(G)
    return r, [None] + [r.pedigree(g) for g in range(1, G + 1)]


def gens_for(orc, kind, S, interval, want=240):
    return min(want, orc.horizon_gen(kind, S, interval) + 1)


@pytest.mark.parametrize("kind,S,bits,interval", SCHEMES)
def test_bounds_against_true_pedigree(orc, kind, S, bits, interval):
    G = gens_for(orc, kind, S, interval)
    r, ped = run_with_pedigree(orc, kind, S, bits, interval, G, seed=3 + kind)
    t, c, s = r.agents()
    lb, ub = orc.mrca_allpairs(kind, S, c, s, bits=bits, interval=interval)
    L = r.layout()
    keep = L != 0xFFFFFFFF
    order = np.argsort(L.astype(np.int64))
    order = [k for k in order if keep[k]]
    times = [int(L[k]) for k in order]
    assert all(tm % interval == 0 for tm in times)
    lines = [lineage(ped, G, a) for a in range(r.A)]
    checked = 0
    for a in range(r.A):
        # against itself: ub = T; lb = 1 + the last deposit (T with no coarsening)
        assert ub[a, a] == G and lb[a, a] == max(times) + 1
        for b in range(r.A):
            assert lb[a, b] == lb[b, a] and ub[a, b] == ub[b, a] and lb[a, b] <= ub[a, b]
            gstar = next((g for g in range(G, -1, -1) if lines[a][g] == lines[b][g]), None)
            if gstar is None:
                continue
            checked += 1
            assert ub[a, b] >= gstar
            tstar = next((tm for k, tm in zip(order, times)
                          if value(s[a], k, bits) != value(s[b], k, bits)), None)
            assert ub[a, b] == (tstar if tstar is not None else G)
            for k, tm in zip(order, times):
                if tm < gstar:
                    assert value(s[a], k, bits) == value(s[b], k, bits)
            end = tstar if tstar is not None else G + 1
            chance = any(gstar <= tm < end for tm in times)
            assert (lb[a, b] <= gstar) == (not chance)
    assert checked > 0


@pytest.mark.parametrize("kind,S,bits,interval", SCHEMES)
def test_retained_values_are_the_ancestors_draws(orc, kind, S, bits, interval):
    G = gens_for(orc, kind, S, interval, 150)
    r, ped = run_with_pedigree(orc, kind, S, bits, interval, G, seed=9)
    _, _, s = r.agents()
    L = r.layout()
    for a in range(r.A):
        anc = lineage(ped, G, a)
        for k in range(S):
            if L[k] == 0xFFFFFFFF:
                continue
            item = int(L[k])
            want = int(ped[item + 1][1][anc[item + 1]])
            assert value(s[a], k, bits) == want, (a, k, item)


@pytest.mark.parametrize("kind,S,bits,interval", [(1, 32, 1, 3), (0, 8, 8, 4), (2, 64, 1, 2)])
def test_only_ingest_generations_write(orc, kind, S, bits, interval):
    r = orc.Run(3, 2, 8, S, kind, seed=5, pedigree_gens=60, bits=bits, interval=interval,
                migrants=0)
    prev = r.agents()[2].copy()
    for g in range(60):
        r.step(1)
        par = r.pedigree(g + 1)[0]
        cur = r.agents()[2]
        parent = prev[par]
        if g % interval:
            assert np.array_equal(cur, parent), g
        else:
            diff = np.nonzero((cur ^ parent).reshape(len(cur), -1).any(axis=0))[0]
            # only the word holding this generation's site can change
            assert len(diff) <= 1
        prev = cur.copy()


def test_horizon_in_generations(orc):
    # tilted, 4 one-byte sites: items up to local time 2^4 - 2 = 14 fit
    for interval in (1, 3):
        last = orc.horizon_gen(1, 4, interval)
        assert last == interval * 15 - 1
        r = orc.Run(2, 2, 4, 4, 1, bits=8, interval=interval)
        r.step(last + 1)
        with pytest.raises(RuntimeError):
            r.step(1)


def test_hand_worked_many_way_tree(orc):
    """Five annotations of four one-byte sites in the fill phase (site k
    holds item k), counter T = 4: (1,1,1,1), (1,2,1,1), (1,3,5,5), (1,3,5,6),
    (7,0,0,0).  The root at t0 = 0 splits off the last; a node at t1 = 1
    splits three ways; a node at t3 = 3 splits the third and fourth."""
    rows = [(1, 1, 1, 1), (1, 2, 1, 1), (1, 3, 5, 5), (1, 3, 5, 6), (7, 0, 0, 0)]
    surf = np.array([[v[0] | v[1] << 8 | v[2] << 16 | v[3] << 24] for v in rows], np.uint32)
    counters = np.full(5, 4, np.uint32)
    sbl, pairs, root, internal, ed = orc.phylo_metrics(0, 4, counters, surf, bits=8)
    assert sbl == 4 + 1 + 3 + 3 + 2 + 1 + 1
    assert pairs == 4 * 4 + 5 * 3 + 1 * 1
    assert root == 0 and internal == 3
    assert np.allclose(ed, [3.25, 3.25, 2.25, 2.25, 4.0])
    lb, ub = orc.mrca_allpairs(0, 4, counters, surf, bits=8)
    assert (lb[0, 1], ub[0, 1]) == (1, 1)
    assert (lb[2, 3], ub[2, 3]) == (3, 3)
    assert (lb[0, 4], ub[0, 4]) == (0, 0)
    assert (lb[1, 2], ub[1, 2]) == (1, 1)


@pytest.mark.parametrize("kind,S,bits,interval", SCHEMES)
def test_tree_agrees_with_bounds(orc, kind, S, bits, interval):
    G = gens_for(orc, kind, S, interval, 400)
    r = orc.Run(4, 4, 16, S, kind, tournament=0, seed=7, bits=bits, interval=interval)
    r.step(G)
    _, c, s = r.agents()
    idx = orc.sample(7, r.A, 120, G)
    sbl, pairs, root, internal, ed = orc.phylo_metrics(kind, S, c[idx], s[idx], bits=bits,
                                                       interval=interval)
    lb, ub = orc.mrca_allpairs(kind, S, c[idx], s[idx], bits=bits, interval=interval)
    iu = np.triu_indices(len(idx), 1)
    assert pairs == int(np.sum(G - ub[iu].astype(np.int64)))
    assert root == int(ub[iu].min())
    assert abs(ed.sum() - sbl) <= 1e-6 * max(sbl, 1)
    assert 1 <= internal <= len(idx) - 1


def test_bytes_collide_less_than_bits(orc):
    """lb overstates relatedness only through chance agreement, which is
    2^-8 per item for bytes against 1/2 for bits."""
    def overstated(bits, S):
        r, ped = run_with_pedigree(orc, 0, S, bits, 1, 200, seed=12)
        _, c, s = r.agents()
        lb, _ = orc.mrca_allpairs(0, S, c, s, bits=bits)
        lines = [lineage(ped, 200, a) for a in range(r.A)]
        bad = tot = 0
        for a in range(r.A):
            for b in range(a + 1, r.A):
                g = next((g for g in range(200, -1, -1) if lines[a][g] == lines[b][g]), None)
                if g is not None:
                    tot += 1
                    bad += int(lb[a, b] > g)
        return bad / tot
    assert overstated(8, 8) < overstated(1, 64) / 4


def test_founder_tags(orc):
    G = 80
    r = orc.Run(4, 4, 16, 32, 1, tournament=0, seed=31, pedigree_gens=G, fitness_model=2,
                migrants=1)
    tags0 = r.agents()[0].copy()
    assert tags0.max() < 2**16 and len(np.unique(tags0)) > 0.95 * r.A
    assert abs(tags0.mean() / 2**16 - 0.5) < 0.05
    sets = [set(tags0.tolist())]
    prev = tags0
    for g in range(1, G + 1):
        r.step(1)
        cur = r.agents()[0].copy()
        par = r.pedigree(g)[0]
        assert np.array_equal(cur, prev[par])          # inherited unchanged
        sets.append(set(cur.tolist()))
        assert sets[-1] <= sets[-2]                    # clades only disappear
        prev = cur
    assert len(sets[-1]) < len(sets[0])


def test_founder_tags_without_migration_stay_on_their_island(orc):
    r = orc.Run(3, 3, 8, 64, 1, tournament=0, seed=2, fitness_model=2, migrants=0)
    tags0 = r.agents()[0].reshape(9, 8).copy()
    r.step(100)
    tags = r.agents()[0].reshape(9, 8)
    for i in range(9):
        assert set(tags[i].tolist()) <= set(tags0[i].tolist())


def test_clades_are_reconstructed_closer(orc):
    """Clade trial shape (3x3 islands x 32, tilted 64, neutral): pairs of
    the same founding clade get later MRCA bounds than pairs of different
    clades, and fewer clades remain as the run grows longer."""
    counts = []
    for G in (25, 50, 100, 250):
        r = orc.Run(3, 3, 32, 64, 1, tournament=0, seed=17, fitness_model=2)
        r.step(G)
        tags, c, s = r.agents()
        counts.append(len(np.unique(tags)))
        lb, ub = orc.mrca_allpairs(1, 64, c, s)
        same = tags[:, None] == tags[None, :]
        off = ~np.eye(len(tags), dtype=bool)
        if (same & off).any() and (~same).any():
            assert ub[same & off].mean() > ub[~same].mean()
    assert counts == sorted(counts, reverse=True) and counts[-1] < counts[0]


@pytest.mark.parametrize("bad", [dict(bits=4), dict(bits=8, S=32), dict(bits=1, S=8),
                                 dict(interval=0)])
def test_invalid_schemes(orc, bad):
    kw = dict(S=32, bits=1, interval=1)
    kw.update(bad)
    S = kw.pop("S")
    with pytest.raises(ValueError):
        orc.Run(2, 2, 4, S, 0, **kw)


def test_tags_need_neutral_selection(orc):
    with pytest.raises(ValueError):
        orc.Run(2, 2, 4, 32, 0, tournament=2, fitness_model=2)
