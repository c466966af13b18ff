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


# --------------------------------------------------------------------------
# The reconstructed tree itself, as canonical Newick text (children ordered by
# their smallest annotation index, polytomy leaves ascending).

def parse_newick(text):
    """(children, length, leaf) nested tuples; leaf is an int or None."""
    pos = 0

    def node():
        nonlocal pos
        children, leaf = [], None
        if text[pos] == "(":
            pos += 1
            while True:
                children.append(node())
                if text[pos] == ",":
                    pos += 1
                    continue
                assert text[pos] == ")"
                pos += 1
                break
        else:
            start = pos
            while text[pos].isdigit():
                pos += 1
            leaf = int(text[start:pos])
        length = None
        if text[pos] == ":":
            pos += 1
            start = pos
            while text[pos].isdigit():
                pos += 1
            length = int(text[start:pos])
        return (children, length, leaf)

    root = node()
    assert text[pos:] == ";"
    return root


def tree_facts(root, T):
    """Sum of branch lengths, internal nodes, and each leaf's ancestor times."""
    sbl, internal = 0, 0
    anc = {}

    def walk(nd, t_here, path):
        nonlocal sbl, internal
        children, length, leaf = nd
        if leaf is not None:
            anc[leaf] = path
            return
        internal += 1
        for ch in children:
            sbl += ch[1]
            walk(ch, t_here + ch[1], path + [(id(nd), t_here)])

    # the root's time: T minus the path length from the root to any leaf
    depth, nd = 0, root
    while nd[2] is None:
        depth += nd[0][0][1]
        nd = nd[0][0]
    walk(root, T - depth, [])
    return sbl, internal, anc


def test_hand_worked_newick(orc):
    rows = [(0, 0, 0, 0), (0, 0, 0, 1), (0, 1, 0, 0), (1, 0, 0, 0)]
    assert orc.phylo_newick(0, 32, np.full(4, 4, np.uint32),
                            bits_to_words(rows, 32)) == "(((0:1,1:1):2,2:3):1,3:4);"
    rows = [(1, 0, 1), (1, 0, 1), (1, 0, 1), (1, 1, 1)]
    assert orc.phylo_newick(1, 32, np.full(4, 3, np.uint32),
                            bits_to_words(rows, 32)) == "((0:0,1:0,2:0):2,3:2);"
    vals = [(1, 1, 1, 1), (1, 2, 1, 1), (1, 3, 5, 5), (1, 3, 5, 6), (7, 0, 0, 0)]
    surf = np.array([[v[0] | v[1] << 8 | v[2] << 16 | v[3] << 24] for v in vals], np.uint32)
    assert orc.phylo_newick(0, 4, np.full(5, 4, np.uint32), surf,
                            bits=8) == "((0:3,1:3,(2:1,3:1):2):1,4:4);"
    assert orc.phylo_newick(0, 32, np.array([7], np.uint32), np.zeros((1, 1), np.uint32)) == "0;"


@pytest.mark.parametrize("kind,S,bits,interval", [(1, 64, 1, 1), (2, 32, 1, 3), (0, 8, 8, 1)])
def test_newick_agrees_with_metrics_and_bounds(orc, kind, S, bits, interval):
    r = orc.Run(4, 4, 16, S, kind, tournament=0, seed=13, bits=bits, interval=interval)
    G = min(500, orc.horizon_gen(kind, S, interval) + 1)
    r.step(G)
    _, c, s = r.agents()
    idx = orc.sample(13, r.A, 80, G)
    text = orc.phylo_newick(kind, S, c[idx], s[idx], bits=bits, interval=interval)
    sbl, pairs, root, internal, _ = orc.phylo_metrics(kind, S, c[idx], s[idx], bits=bits,
                                                      interval=interval)
    t_sbl, t_internal, anc = tree_facts(parse_newick(text), G)
    assert (t_sbl, t_internal) == (sbl, internal)
    assert sorted(anc) == list(range(len(idx)))
    lb, ub = orc.mrca_allpairs(kind, S, c[idx], s[idx], bits=bits, interval=interval)
    for a in range(len(idx)):
        for b in range(a + 1, len(idx)):
            shared = [t for (na, t), (nb, _) in zip(anc[a], anc[b]) if na == nb]
            assert shared[-1] == ub[a, b]       # the MRCA sits at the upper bound
