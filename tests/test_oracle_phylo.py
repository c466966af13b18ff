"""Pins of the oracle's trie reconstruction and phylometrics (Distributed
Phylogenetic Tracking: reconstruction is a trie-building procedure over the
record of differentiae; Results, On-hardware Trial: sum branch length and
mean evolutionary distinctiveness separate treatments).

* a hand-worked four-leaf tree;
* fair-proportion evolutionary distinctiveness sums to the tree length;
* every pair's MRCA in the tree sits at the pair's MRCA upper bound, so the
  pairwise sum equals the sum of (T - ub) from the (pinned) bounds;
* identical annotations form a polytomy at T; one annotation is a lone
  leaf; differing counters are refused.
"""
import numpy as np
import pytest


def bits_to_words(bit_rows, S):
    """Annotations given as bits in site order (fill phase: site k = item k)."""
    out = np.zeros((len(bit_rows), S // 32), np.uint32)
    for a, row in enumerate(bit_rows):
        for k, b in enumerate(row):
            out[a, k // 32] |= np.uint32(b) << np.uint32(k % 32)
    return out


def test_hand_worked_tree(orc):
    # steady, S = 32, T = 4: site k holds item k; bits in time order
    rows = [(0, 0, 0, 0), (0, 0, 0, 1), (0, 1, 0, 0), (1, 0, 0, 0)]
    surf = bits_to_words(rows, 32)
    sbl, pairs, root, internal, ed = orc.phylo_metrics(0, 32, np.full(4, 4, np.uint32), surf)
    # root at t0 = 0 splits {a,b,c} | d; node at 1 splits {a,b} | c; node at 3 splits a | b
    assert sbl == 4 + 1 + 3 + 2 + 1 + 1
    assert pairs == 3 * 4 + 2 * (4 - 1) + 1 * (4 - 3)
    assert root == 0 and internal == 3
    assert np.allclose(ed, [1 / 3 + 1 + 1, 1 / 3 + 1 + 1, 1 / 3 + 3, 4])


def test_polytomy_of_identical_annotations(orc):
    rows = [(1, 0, 1), (1, 0, 1), (1, 0, 1), (1, 1, 1)]
    surf = bits_to_words(rows, 32)
    sbl, pairs, root, internal, ed = orc.phylo_metrics(1, 32, np.full(4, 3, np.uint32), surf)
    # root at t1 = 1 splits {three identical} | other; the three hang from a node at T = 3
    assert root == 1 and internal == 2
    assert sbl == (3 - 1) + (3 - 1)
    assert pairs == 3 * 1 * (3 - 1)
    assert np.allclose(ed, [2 / 3, 2 / 3, 2 / 3, 2])


def test_single_and_refused(orc):
    surf = np.zeros((1, 1), np.uint32)
    assert orc.phylo_metrics(0, 32, np.array([7], np.uint32), surf)[:4] == (0, 0, 7, 0)
    with pytest.raises(ValueError):
        orc.phylo_metrics(0, 32, np.array([7, 8], np.uint32), np.zeros((2, 1), np.uint32))


@pytest.mark.parametrize("kind", [0, 1, 2])
@pytest.mark.parametrize("tournament", [0, 2])
def test_tree_agrees_with_bounds_and_identity(orc, kind, tournament):
    r = orc.Run(4, 4, 16, 64, kind, tournament=tournament, seed=3 + kind)
    r.step(700)
    t, c, s = r.agents()
    idx = orc.sample(r.seed, r.A, 96, 700)
    sbl, pairs, root, internal, ed = orc.phylo_metrics(kind, 64, c[idx], s[idx])
    lb, ub = orc.mrca_allpairs(kind, 64, c[idx], s[idx])
    iu = np.triu_indices(len(idx), 1)
    assert pairs == int(np.sum(700 - ub[iu].astype(np.int64)))
    assert root == int(ub[iu].min())
    assert abs(ed.sum() - sbl) <= 1e-6 * max(sbl, 1)
    assert 1 <= internal <= len(idx) - 1
    # every leaf edge ends at T; no branch is negative
    assert sbl >= 700 - root


def test_selection_shortens_the_tree(orc):
    """Selective sweeps make common ancestry recent: a shorter tree."""
    vals = {}
    for tour in (2, 0):
        r = orc.Run(8, 8, 32, 64, 1, tournament=tour, seed=1)
        r.step(3000)
        t, c, s = r.agents()
        idx = orc.sample(1, r.A, 256, 3000)
        vals[tour] = orc.phylo_metrics(1, 64, c[idx], s[idx])[0]
    assert vals[2] < vals[0]
