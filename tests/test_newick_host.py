"""The library's host Newick formatter (hstrat_phylo_newick) on hand-built
trees: canonical order (children by the smallest annotation index below
them), branch lengths as parent-to-child time differences, leaves at T,
polytomies at T with zero-length leaf edges, and refused malformed trees.
No GPU is needed."""
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2404_10861_amd", "libhsga.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libhsga.so not built")
R, X = 0xFFFFFFFF, 0xFFFFFFFE


def tree(leaf, npar, ntime, T):
    return {"leaf_parent": np.array(leaf, np.uint32), "node_parent": np.array(npar, np.uint32),
            "node_time": np.array(ntime, np.uint32), "T": T}


def test_hand_built_trees():
    import paper_2404_10861_amd as hs
    # root (boundary 1, time 2) over node 0 (time 5: leaves 0, 1) and leaves 2, 3
    assert hs.newick(tree([0, 0, 1, 1], [1, R, X], [5, 2, 0], 10)) == "((0:5,1:5):3,2:8,3:8);"
    # a polytomy of identical annotations: a node at T, zero-length leaves
    assert hs.newick(tree([0, 0, 0], [R, X], [12, 0], 12)) == "(0:0,1:0,2:0);"
    assert hs.newick(tree([R], [], [], 7)) == "0;"


def test_canonical_order_and_lengths():
    import paper_2404_10861_amd as hs
    # root 0 (time 1) over node 2 (time 4: leaves 3, 1) and node 1 (time 6: leaves 0, 2)
    t = tree([1, 2, 1, 2], [R, 0, 0], [1, 6, 4], 10)
    assert hs.newick(t) == "((0:4,2:4):5,(1:6,3:6):3);"


def test_malformed_trees_are_refused():
    import paper_2404_10861_amd as hs
    with pytest.raises(hs.HsgaError):
        hs.newick(tree([0, 0, 5], [R, X], [1, 0], 3))          # leaf parent out of range
    with pytest.raises(hs.HsgaError):
        hs.newick(tree([0, 0, 1], [R, R], [1, 1], 3))          # two roots
    with pytest.raises(hs.HsgaError):
        hs.newick(tree([0, 0, 1], [1, 0], [1, 1], 3))          # no root (a cycle)
    # a root, and boundaries 2 and 3 parenting each other apart from it
    with pytest.raises(hs.HsgaError):
        hs.newick(tree([0, 0, 2, 3, 0], [R, 0, 3, 2], [1, 2, 2, 2], 5))
    # a leaf hanging from a boundary that names no node
    with pytest.raises(hs.HsgaError):
        hs.newick(tree([0, 0, 1], [R, X], [1, 0], 3))
    # a node older than its parent; a node younger than the leaves
    with pytest.raises(hs.HsgaError):
        hs.newick(tree([0, 1, 1], [R, 0], [4, 2], 9))
    with pytest.raises(hs.HsgaError):
        hs.newick(tree([0, 1, 1], [R, 0], [4, 12], 9))
    # the same shapes, well formed, are accepted
    assert hs.newick(tree([0, 1, 1], [R, 0], [2, 4], 9)) == "(0:7,(1:5,2:5):2);"
