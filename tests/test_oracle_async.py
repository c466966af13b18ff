"""Pins of the oracle's asynchronous runs (Methods, Asynchronous
Island-model Genetic Algorithm: islands run their own generation loops and
drift apart): with every island active on every tick it is the synchronous
run; inactive islands stay as they are and post nothing; every birth
raises its parent's own counter by one and deposits at the site the rule
gives that counter; the MRCA bounds of agents with different counters hold
against the true pedigree; islands drift apart."""
import numpy as np
import pytest

ALL = 0xFFFFFFFF


def value(s, k, bits):
    per = 32 // bits
    return (int(s[k // per]) >> ((k % per) * bits)) & ((1 << bits) - 1)


def history(orc, K, **kw):
    """Run K ticks one at a time: per tick the agents and the pedigree."""
    r = orc.Run(pedigree_gens=K, **kw)
    states = [tuple(x.copy() for x in r.agents())]
    outs = [None]
    for _ in range(K):
        r.step(1)
        states.append(tuple(x.copy() for x in r.agents()))
        outs.append(r.outbox())
    ped = [None] + [r.pedigree(k)[0] for k in range(1, K + 1)]
    return r, states, outs, ped


def base(**kw):
    d = dict(W=4, H=3, N=8, S=32, kind=1, seed=5)
    d.update(kw)
    return d


@pytest.mark.parametrize("kw", [dict(), dict(kind=2, S=64, tournament=0),
                                dict(kind=0, S=8, bits=8, interval=3),
                                dict(fitness_model=1, tournament=5, del_thr=1417339207,
                                     ben_thr=12884901),
                                dict(fitness_model=2, tournament=0, migrants=1)])
def test_all_active_is_the_synchronous_run(orc, kw):
    cfg = base(**kw)
    K = 150
    # the activity draws of this window are all below the threshold
    for k in range(K):
        for i in range(cfg["W"] * cfg["H"]):
            assert orc.philox(0, i, k, orc.ACTIVITY, cfg["seed"])[0] < ALL
    a = orc.Run(activity=ALL, **cfg)
    b = orc.Run(**cfg)
    a.step(K)
    b.step(K)
    for x, y in zip(a.agents(), b.agents()):
        assert np.array_equal(x, y)
    assert np.array_equal(a.layout(), b.layout())
    for x, y in zip(a.outbox(), b.outbox()):
        assert np.array_equal(x, y)


def test_inactive_islands_stay_and_post_nothing(orc):
    p = int(0.6 * 2**32)
    cfg = base(activity=p, migrants=1)
    K = 80
    r, states, outs, ped = history(orc, K, **cfg)
    I, N = 12, 8
    active_count = 0
    for k in range(K):
        for i in range(I):
            act = orc.philox(0, i, k, orc.ACTIVITY, 5)[0] < p
            active_count += act
            sl = slice(i * N, (i + 1) * N)
            if not act:
                for x, y in zip(states[k], states[k + 1]):
                    assert np.array_equal(x[sl], y[sl])
                assert outs[k + 1][0][i] == 4          # no emigrant
            else:
                assert outs[k + 1][0][i] < 4
    n = K * I
    assert abs(active_count - 0.6 * n) < 5 * np.sqrt(n * 0.24)


def test_births_raise_the_parents_own_counter(orc):
    cfg = base(activity=int(0.7 * 2**32), migrants=1)
    K = 120
    r, states, outs, ped = history(orc, K, **cfg)
    for k in range(K):
        c0, c1 = states[k][1], states[k + 1][1]
        par = ped[k + 1]
        for a in range(len(c1)):
            born = c1[a] != c0[par[a]] or par[a] != a
            if born:
                assert c1[a] == c0[par[a]] + 1
            else:
                assert c1[a] == c0[a]
        assert c1.max() <= k + 1
    # drift: the counters of one island differ
    assert max(len(np.unique(states[K][1][i * 8:(i + 1) * 8])) for i in range(12)) > 1


def test_immigrants_come_from_active_neighbours(orc):
    p = int(0.5 * 2**32)
    cfg = base(activity=p, migrants=1, W=5, H=4)
    K = 60
    r, states, outs, ped = history(orc, K, **cfg)
    W, H, N = 5, 4, 8
    for k in range(1, K):
        for a, src in enumerate(ped[k + 1]):
            i, si = a // N, int(src) // N
            if si == i:
                continue
            # a parent from another island: an emigrant that island posted
            # on the previous tick, i.e. it was active then
            assert orc.philox(0, si, k - 1, orc.ACTIVITY, 5)[0] < p
            assert orc.philox(0, i, k, orc.ACTIVITY, 5)[0] < p
            x, y = i % W, i // W
            nbrs = {((x) % W) + ((y - 1) % H) * W, (x % W) + ((y + 1) % H) * W,
                    ((x - 1) % W) + y * W, ((x + 1) % W) + y * W}
            assert si in nbrs


@pytest.mark.parametrize("kind,S,bits,interval", [(1, 32, 1, 1), (2, 64, 1, 3), (0, 8, 8, 2)])
def test_retained_values_follow_each_agents_counter(orc, kind, S, bits, interval):
    cfg = base(activity=int(0.65 * 2**32), migrants=1, kind=kind, S=S, bits=bits,
               interval=interval)
    K = min(160, orc.horizon_gen(kind, S, interval) + 1)
    r, states, outs, ped = history(orc, K, **cfg)
    _, c, s = states[K]
    pb = [None] + [r.pedigree(k)[1] for k in range(1, K + 1)]
    for a in range(len(c)):
        # walk back: anc[k] = index at tick k; find the birth that gave each counter
        anc = {K: a}
        for k in range(K, 0, -1):
            anc[k - 1] = int(ped[k][anc[k]])
        drawn = {}
        for k in range(K):
            before = states[k][1][anc[k]]
            after = states[k + 1][1][anc[k + 1]]
            if after == before + 1:
                drawn[int(after)] = int(pb[k + 1][anc[k + 1]])
        L = orc.layout(kind, S, -(-int(c[a]) // interval))
        for site in range(S):
            if L[site] == 0xFFFFFFFF:
                continue
            t = int(L[site]) * interval
            assert value(s[a], site, bits) == drawn[t + 1], (a, site, t)


def test_bounds_with_drifting_counters_against_the_pedigree(orc):
    cfg = base(activity=int(0.7 * 2**32), migrants=1, kind=2, S=64, W=3, H=2, N=4)
    K = 200
    r, states, outs, ped = history(orc, K, **cfg)
    t, c, s = states[K]
    assert len(np.unique(c)) > 1
    lb, ub = orc.mrca_allpairs(2, 64, c, s)
    A = len(c)
    lines = []
    for a in range(A):
        anc = {K: a}
        for k in range(K, 0, -1):
            anc[k - 1] = int(ped[k][anc[k]])
        lines.append(anc)
    checked = 0
    for a in range(A):
        for b in range(A):
            kstar = next((k for k in range(K, -1, -1) if lines[a][k] == lines[b][k]), None)
            if kstar is None:
                continue
            gstar = int(states[kstar][1][lines[a][kstar]])   # the MRCA's counter
            checked += 1
            assert ub[a, b] >= gstar
            assert lb[a, b] <= ub[a, b]
    assert checked > 0


def test_async_needs_a_fresh_run(orc):
    r = orc.Run(2, 2, 4, 32, 0)
    r.step(1)
    assert orc.load().orc_set_async(r._h, 5) != 0
