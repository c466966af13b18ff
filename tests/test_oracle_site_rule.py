"""Brute-force pins of the oracle's surface site rule.

The paper fixes properties of the surface, not the indexing algorithm
(Methods, Distributed Phylogenetic Tracking and Surface-based Hereditary
Stratigraphy Algorithms):

* one fixed-width buffer; each generation writes one site; items stay where
  they were written until overwritten;
* timestamps follow from the site index and the elapsed generation count;
* steady policy: retained time points spread evenly over history;
* tilted policy: recent time points are preferred;
* hybrid: half of the space to each policy.

Every T up to the horizon is replayed for small surfaces (m = 4, 8, 16
sites), and each layout is checked against those properties made
quantitative, plus the retention target D(T) enumerated constructively here
(not through the oracle's membership test):

* steady: D(T) = multiples of g(T) = 2^bitlen(floor(T/(m-1))), plus T;
  the earliest item 0 stays; consecutive retained items are at most g(T)
  apart, and g(T) <= max(1, 2T/(m-1)) (even spread within a factor 2);
* tilted: on each level h (t+1 = (2c+1) 2^h) the r = floor(m/bitlen(T+1))
  most recent items; T itself stays; consecutive retained items a < b are
  at most about 2(T-b)/(2r-1) apart (gap proportional to age).
"""
import numpy as np
import pytest

EMPTY = 0xFFFFFFFF


def bitlen(x):
    return int(x).bit_length()


def steady_target(m, T):
    g = 1 << bitlen(T // (m - 1))
    D = set(range(0, T + 1, g))
    D.add(T)
    return D, g


def tilted_target(m, T):
    B = bitlen(T + 1)
    r = m // B
    D = set()
    for h in range(B):
        n_h = (T + 1 + (1 << h)) >> (h + 1)      # level-h items up to T
        for c in range(max(0, n_h - r), n_h):
            D.add((2 * c + 1) * (1 << h) - 1)
    return D, r


def replay_checked(orc, kind, m, T_end, check):
    """Ingest items 0..T_end one at a time; call check(T, site, layout)."""
    L = np.full(m, EMPTY, np.uint32)
    for T in range(T_end + 1):
        site = orc.place(kind, m, L, T)
        assert 0 <= site < m, (T, site)
        if T < m:
            assert site == T, "fill phase writes site T"
        else:
            assert L[site] != EMPTY
        L[site] = T
        check(T, site, L)
    return L


@pytest.mark.parametrize("m", [4, 8, 16])
def test_steady_criteria(orc, m):
    T_end = (1 << m) - 1 if m < 16 else (1 << 16) - 1

    def check(T, site, L):
        held = L[L != EMPTY].astype(np.int64)
        assert len(np.unique(held)) == len(held)
        assert held.max() == T
        D, g = steady_target(m, T)
        assert len(D) == T // g + 1 + (1 if T % g else 0)   # closed-form count
        assert len(D) <= m
        assert D.issubset(set(held.tolist())), T
        s = np.sort(held)
        assert s[0] == 0, "the earliest item is kept"
        if len(s) > 1:
            gap = int(np.max(np.diff(s)))
            assert gap <= g
        assert g <= max(1, 2 * T / (m - 1))
    replay_checked(orc, 0, m, T_end, check)


@pytest.mark.parametrize("m", [4, 8, 16])
def test_tilted_criteria(orc, m):
    T_end = (1 << m) - 2           # last T with r >= 1

    def check(T, site, L):
        held = L[L != EMPTY].astype(np.int64)
        assert len(np.unique(held)) == len(held)
        D, r = tilted_target(m, T)
        assert r >= 1
        B = bitlen(T + 1)
        count = sum(min(r, (T + 1 + (1 << h)) >> (h + 1)) for h in range(B))
        assert len(D) == count <= m
        assert T in D
        assert D.issubset(set(held.tolist())), T
        s = np.sort(held)
        a, b = s[:-1], s[1:]
        lhs = (b - a) * (2 * r - 1)
        rhs = np.maximum(2 * r - 1, 2 * (T - b))
        assert np.all(lhs <= rhs), T
    replay_checked(orc, 1, m, T_end, check)


@pytest.mark.parametrize("S", [32, 64])
def test_hybrid_is_half_steady_half_tilted(orc, S):
    m = S // 2
    n = 6000
    hyb = orc.site_sequence(2, S, 0, n)
    st = orc.site_sequence(0, m, 0, n // 2)
    ti = orc.site_sequence(1, m, 0, n // 2)
    assert np.array_equal(hyb[0::2], st)
    assert np.array_equal(hyb[1::2], ti + m)


@pytest.mark.parametrize("kind", [0, 1, 2])
@pytest.mark.parametrize("S", [32, 64])
def test_layout_replay_matches_incremental(orc, kind, S):
    """Timestamps from (site, elapsed generations) alone: the layout replayed
    from scratch for T equals the one built incrementally."""
    L = np.full(S, EMPTY, np.uint32)
    for T in range(3000):
        if T % 97 == 0 or T < 70:
            assert np.array_equal(orc.layout(kind, S, T), L), T
        L[orc.place(kind, S, L, T)] = T


@pytest.mark.parametrize("S", [32, 64])
def test_large_surface_invariants(orc, S):
    """S = 32 and 64 (the configured sizes): full surface after the fill
    phase, the target retained, for T up to 20,000."""
    for kind in (0, 1):
        L = np.full(S, EMPTY, np.uint32)
        for T in range(20001):
            L[orc.place(kind, S, L, T)] = T
            if T >= S - 1 and T % 251 == 0:
                assert np.all(L != EMPTY)
                D, _ = (steady_target if kind == 0 else tilted_target)(S, T)
                assert D.issubset(set(L.tolist()))


def test_horizon(orc):
    # tilted: T <= 2^S - 2 keeps r >= 1; the 32-bit counter caps at 2^32 - 2
    assert orc.horizon(1, 32) == 2**32 - 2
    assert orc.horizon(1, 64) == 2**32 - 2
    assert orc.horizon(0, 32) == 2**32 - 2
    # hybrid S = 32: 16-site tilted half, local u <= 2^16 - 2, T = 2u + 1
    h = orc.horizon(2, 32)
    assert h == 2 * (2**16 - 2) + 2
    assert bitlen((h - 1) // 2 + 1) <= 16          # last odd T is inside
    assert bitlen((h + 1 - 1) // 2 + 1) > 16       # next odd T is outside
    assert orc.horizon(2, 64) == 2**32 - 2
    # a small tilted surface really runs out at its horizon
    m = 4
    T_h = 2**m - 2
    assert m // bitlen(T_h + 1) >= 1 and m // bitlen(T_h + 2) == 0


def test_site_rule_is_one_write_per_generation_over_a_long_run(orc):
    seq = orc.site_sequence(1, 32, 0, 20000)
    assert seq.min() >= 0 and seq.max() < 32
    assert np.array_equal(seq[:32], np.arange(32))


@pytest.mark.parametrize("kind,S", [(1, 4), (1, 8), (2, 8), (2, 16), (1, 16)])
def test_no_placement_past_the_horizon(orc, kind, S):
    """The retention target is defined up to the horizon only: the last
    placeable item is the horizon itself; the next one, and a layout that
    would hold it, are refused rather than placed."""
    h = orc.horizon(kind, S)
    L = orc.layout(kind, S, h + 1)                  # items 0 .. h
    assert orc.place(kind, S, L, h + 1) == -1
    with pytest.raises(ValueError):
        orc.layout(kind, S, h + 2)
    with pytest.raises(ValueError):
        orc.site_sequence(kind, S, h - 2, 4)
    assert len(orc.site_sequence(kind, S, h - 2, 3)) == 3
    # the queries (byte differentiae: 4 or 8 sites) refuse annotations whose
    # counter holds such an item
    if S * 8 not in (32, 64):
        return
    c_ok = np.full(3, h + 1, np.uint32)
    surf = np.zeros((3, S * 8 // 32), np.uint32)
    orc.mrca_allpairs(kind, S, c_ok, surf, bits=8)
    orc.phylo_metrics(kind, S, c_ok, surf, bits=8)
    with pytest.raises(ValueError):
        orc.mrca_allpairs(kind, S, c_ok + 1, surf, bits=8)
    with pytest.raises(ValueError):
        orc.phylo_metrics(kind, S, c_ok + 1, surf, bits=8)
