"""Placement vectors of the site rule, worked out from the reading (fill the
sub-surface in order, then overwrite the lowest site whose item left the
retention target) independently of the oracle and of the kernels
(Methods, Surface-based Hereditary Stratigraphy Algorithms; the first
entries are derived by hand in the fixture's header).

The brute-force criteria of test_oracle_site_rule.py hold for any choice
among the evictable sites; these vectors pin the choice itself.
"""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def load_vectors():
    rows = []
    with open(os.path.join(HERE, "golden", "site_rule_vectors.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            head, values = line.split(":")
            name, kind, S, T0 = head.split()
            rows.append((name, int(kind), int(S), int(T0),
                         np.array([int(v) for v in values.split()], np.int64)))
    return rows


def test_fixture_has_the_six_vectors():
    rows = load_vectors()
    assert [(r[0], r[1], r[2]) for r in rows] == [
        ("seq", 0, 8), ("seq", 1, 8), ("seq", 0, 32), ("seq", 1, 32),
        ("layout", 0, 32), ("layout", 1, 32)]


def test_vectors_match_oracle(orc):
    for name, kind, S, T0, want in load_vectors():
        if name == "seq":
            got = orc.site_sequence(kind, S, T0, len(want))
        else:
            got = orc.layout(kind, S, T0)
        assert np.array_equal(np.asarray(got, np.int64), want), (name, kind, S, T0)


def test_hybrid_halves_follow_the_vectors(orc):
    """A hybrid-64 surface runs the 32-site steady rule on even generations
    (sites 0..31) and the 32-site tilted rule on odd ones (sites 32..63)."""
    rows = {(r[0], r[1], r[2], r[3]): r[4] for r in load_vectors()}
    seq = orc.site_sequence(2, 64, 64, 64)          # local times 32..63
    assert np.array_equal(seq[0::2], rows[("seq", 0, 32, 32)])
    assert np.array_equal(seq[1::2] - 32, rows[("seq", 1, 32, 32)])
    L = orc.layout(2, 64, 2000)                     # 1,000 ingests per half
    assert np.array_equal(L[:32] // 2, rows[("layout", 0, 32, 1000)])
    assert np.array_equal((L[32:] - 1) // 2, rows[("layout", 1, 32, 1000)])
