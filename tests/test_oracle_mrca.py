"""Pins of the oracle's MRCA-generation bounds and end-of-run sampling.

Mismatching differentiae delimit the extent of common ancestry, and one-bit
differentiae can collide and make lineages look more related than they are
(Methods, Distributed Phylogenetic Tracking; Results, Clade Reconstruction
Trial).  On tiny runs the true pedigree is known, so for every ordered pair
with a most recent common ancestor at generation g*:

* ub >= g* always (a mismatch can only arise after the lineages split);
* every retained item older than g* agrees (inherited from the ancestor);
* lb <= g* exactly when no commonly retained item t with g* <= t < t*
  (t* the first mismatch) agreed by chance, the collision case;
* an agent against itself gives (T, T); founders give (0, 0).

Hand-built annotations pin the bound arithmetic on the fill phase, where
site k holds item k.
"""
import numpy as np
import pytest


def bit(s, k):
    return (int(s[k // 32]) >> (k % 32)) & 1


def lineage(ped, G, a):
    anc = {G: a}
    for g in range(G, 0, -1):
        anc[g - 1] = int(ped[g][0][anc[g]])
    return anc


@pytest.mark.parametrize("kind", [0, 1, 2])
@pytest.mark.parametrize("S", [32, 64])
@pytest.mark.parametrize("tournament", [0, 2])
def test_bounds_against_true_pedigree(orc, kind, S, tournament):
    W, H, N, G = 2, 2, 4, 300
    r = orc.Run(W, H, N, S, kind, tournament=tournament, seed=1 + kind,
                pedigree_gens=G)
    r.step(G)
    ped = [None] + [r.pedigree(g) for g in range(1, G + 1)]
    t, c, s = r.agents()
    lb, ub = orc.mrca_allpairs(kind, S, c, s)
    L = r.layout()
    order = np.argsort(L.astype(np.int64))
    times = L[order].astype(np.int64)
    lines = [lineage(ped, G, a) for a in range(r.A)]
    collisions = 0
    checked = 0
    for a in range(r.A):
        assert lb[a, a] == G and ub[a, a] == G
        for b in range(r.A):
            assert lb[a, b] == lb[b, a] and ub[a, b] == ub[b, a]
            assert lb[a, b] <= ub[a, b]
            gstar = None
            for g in range(G, -1, -1):
                if lines[a][g] == lines[b][g]:
                    gstar = g
                    break
            if gstar is None:
                continue               # lineages from different founders
            checked += 1
            assert ub[a, b] >= gstar
            tstar = None
            for k, tm in zip(order, times):
                if bit(s[a], k) != bit(s[b], k):
                    tstar = tm
                    break
            for k, tm in zip(order, times):
                if tm < gstar:
                    assert bit(s[a], k) == bit(s[b], k)
            end = tstar if tstar is not None else G + 1
            chance = any(gstar <= tm < end for tm in times)
            assert (lb[a, b] <= gstar) == (not chance)
            collisions += int(chance)
    assert checked > 0
    assert collisions > 0 or tournament == 2


def test_founders_give_zero_bounds(orc):
    for kind in (0, 1, 2):
        z = np.zeros((3, 2), np.uint32)
        lb, ub = orc.mrca_allpairs(kind, 64, np.zeros(3, np.uint32), z)
        assert np.all(lb == 0) and np.all(ub == 0)


def test_hand_built_fill_phase_annotations(orc):
    # steady, S = 32, T = 10: site k holds item k for k < 10
    sa = np.zeros(1, np.uint32)
    sb = np.zeros(1, np.uint32)
    sa[0] = 0b0000011111
    sb[0] = 0b0000001111      # first difference at item 4
    assert orc.mrca_pair(32, 10, sa, 10, sb, 0) == (4, 4)
    sb[0] = 0b0000011110      # first difference at item 0
    assert orc.mrca_pair(32, 10, sa, 10, sb, 0) == (0, 0)
    # identical: the last common item 9 agrees -> (10, 10)
    assert orc.mrca_pair(32, 10, sa, 10, sa, 0) == (10, 10)
    # different generation counts: items 0..9 common; no mismatch
    sc = np.array([0b110000011111], np.uint32)
    assert orc.mrca_pair(32, 10, sa, 12, sc, 0) == (10, 10)
    # differ only in item 11, which the younger one lacks
    sd = np.array([0b010000011111], np.uint32)
    assert orc.mrca_pair(32, 12, sc, 12, sd, 0) == (11, 11)
    # differ in item 10: items 0..9 agree
    se = np.array([0b100000011111], np.uint32)
    assert orc.mrca_pair(32, 12, sc, 12, se, 0) == (10, 10)


def test_bounds_with_unequal_counters_match_pairwise(orc):
    """All-pairs over annotations of different ages equals the pair form."""
    rng = np.random.default_rng(3)
    for kind in (0, 1, 2):
        counters = np.array([0, 5, 33, 100, 100, 257, 1000], np.uint32)
        surf = rng.integers(0, 2**32, size=(len(counters), 2), dtype=np.uint64)
        surf = surf.astype(np.uint32)
        lb, ub = orc.mrca_allpairs(kind, 64, counters, surf)
        for a in range(len(counters)):
            for b in range(len(counters)):
                pl, pu = orc.mrca_pair(64, int(counters[a]), surf[a],
                                       int(counters[b]), surf[b], kind)
                assert (lb[a, b], ub[a, b]) == (pl, pu)
                assert ub[a, b] <= min(counters[a], counters[b])


def test_rows_equal_allpairs(orc):
    rng = np.random.default_rng(8)
    counters = np.full(40, 500, np.uint32)
    counters[5:9] = [0, 17, 499, 501]
    surf = rng.integers(0, 2**32, size=(40, 2), dtype=np.uint64).astype(np.uint32)
    lb, ub = orc.mrca_allpairs(2, 64, counters, surf)
    rows = [0, 6, 39, 7, 7]
    rlb, rub = orc.mrca_rows(2, 64, counters, surf, rows)
    assert np.array_equal(rlb, lb[rows]) and np.array_equal(rub, ub[rows])


@pytest.mark.parametrize("A,n", [(2048, 1024), (4194304, 4096), (1000, 1000),
                                 (500, 1024), (7, 3)])
def test_stratified_sample(orc, A, n):
    idx = orc.sample(5, A, n, 123)
    if A <= n:
        assert np.array_equal(idx, np.arange(A))
        return
    assert len(idx) == n
    k = np.arange(n, dtype=np.int64)
    lo = k * A // n
    hi = (k + 1) * A // n
    assert np.all(idx >= lo) and np.all(idx < hi)
    assert np.all(np.diff(idx.astype(np.int64)) > 0)
    other = orc.sample(5, A, n, 124)
    assert not np.array_equal(idx, other) or n < 4
