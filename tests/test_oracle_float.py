"""Pins of the oracle's float treatments (Results, On-hardware Trial;
Asynchronous Island-model Genetic Algorithm): the half-normal draw against
the exact function at 50 digits and against its law; the tournament's rank
law; the sign, frequency and size of deleterious and beneficial mutations
read from the pedigree; ties and one-draw tournaments reducing to neutral."""
import math

import mpmath
import numpy as np
import pytest
from scipy import stats

F = 1  # float fitness model
P_DEL = int(0.33 * 2**32)
P_BEN = int(0.003 * 2**32)


def exact_half_normal(w1, w2):
    mpmath.mp.dps = 50
    u1 = (mpmath.mpf(w1) + mpmath.mpf(0.5)) / 2**32
    u2 = (mpmath.mpf(w2) + mpmath.mpf(0.5)) / 2**32
    return mpmath.sqrt(-2 * mpmath.log(u1)) * mpmath.cos(mpmath.pi / 2 * u2)


def test_half_normal_exact_to_1e14(orc):
    rng = np.random.default_rng(7)
    edge = [0, 1, 2, 2**31 - 1, 2**31, 2**31 + 1, 2**32 - 2, 2**32 - 1, 0x5A827999, 0xB504F333]
    pairs = [(a, b) for a in edge for b in edge]
    pairs += [tuple(int(x) for x in r) for r in rng.integers(0, 2**32, size=(1500, 2))]
    worst = 0.0
    for w1, w2 in pairs:
        got = orc.half_normal(w1, w2)
        want = exact_half_normal(w1, w2)
        worst = max(worst, float(abs(got - want) / want))
    assert worst < 1e-14


def test_half_normal_law(orc):
    # the birth blocks' radius and angle words of a run: E|Z| = sqrt(2/pi),
    # E Z^2 = 1, and the half-normal CDF
    z = np.array([orc.half_normal(*orc.philox(j, i, 0, orc.BIRTH_B, 99)[2:4])
                  for i in range(1000) for j in range(100)])
    n = z.size
    assert abs(z.mean() - math.sqrt(2 / math.pi)) < 5 * math.sqrt(1 - 2 / math.pi) / math.sqrt(n)
    assert abs((z * z).mean() - 1.0) < 5 * math.sqrt(2.0) / math.sqrt(n)
    assert stats.kstest(z, stats.halfnorm.cdf).pvalue > 1e-3
    assert z.min() > 0


def gens_with_pedigree(orc, G, **kw):
    base = dict(W=3, H=2, N=16, S=32, kind=2, migrants=0, seed=11, pedigree_gens=G,
                fitness_model=F)
    base.update(kw)
    r = orc.Run(**base)
    fit = [orc.as_f32(r.agents()[0]).copy()]
    for _ in range(G):
        r.step(1)
        fit.append(orc.as_f32(r.agents()[0]).copy())
    ped = [r.pedigree(g + 1)[0] for g in range(G)]   # parents in P_g of P_{g+1}
    return r, fit, ped


def test_no_mutation_keeps_zero_and_ties_reduce_to_one_draw(orc):
    _, fit5, ped5 = gens_with_pedigree(orc, 30, tournament=5, del_thr=0, ben_thr=0)
    _, fit1, ped1 = gens_with_pedigree(orc, 30, tournament=1, del_thr=0, ben_thr=0)
    _, fit0, ped0 = gens_with_pedigree(orc, 30, tournament=0, del_thr=0, ben_thr=0)
    assert all(np.all(f == 0.0) for f in fit5)
    for a, b, c in zip(ped5, ped1, ped0):       # every tie keeps the first draw
        assert np.array_equal(a, b) and np.array_equal(b, c)


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_tournament_rank_law(orc, k):
    """With all fitness values distinct (every birth mutates), the parent's
    rank from the top within its island has P(rank <= r) = 1 - (1 - r/N)^k."""
    N = 16
    _, fit, ped = gens_with_pedigree(orc, 60, tournament=k, del_thr=2**32 - 1, ben_thr=0,
                                     W=4, H=4, N=N)
    counts = np.zeros(N)
    for g in range(5, 60):
        f = fit[g]
        for a, par in enumerate(ped[g]):
            isl = a // N
            fi = f[isl * N:(isl + 1) * N]
            assert par // N == isl
            counts[int(np.sum(fi > f[par]))] += 1
    r = np.arange(N + 1)
    cdf = 1 - (1 - r / N) ** k
    expect = np.diff(cdf) * counts.sum()
    chi2 = float(np.sum((counts - expect) ** 2 / expect))
    assert stats.chi2.sf(chi2, N - 1) > 1e-4, (counts, expect)


def test_mutation_sign_frequency_and_size(orc):
    sig_d, sig_b = 0.5, 2.0
    G = 40
    _, fit, ped = gens_with_pedigree(orc, G, tournament=5, del_thr=P_DEL, ben_thr=P_BEN * 40,
                                     del_sigma=sig_d, ben_sigma=sig_b, W=8, H=8, N=32)
    dn, up, same, total = [], [], 0, 0
    for g in range(G):
        child = fit[g + 1]
        parent = fit[g][ped[g]]
        d = child.astype(np.float64) - parent.astype(np.float64)
        total += d.size
        same += int(np.sum(d == 0))
        if g < 3:     # small |fitness|: binary32 rounding is negligible
            dn += list(-d[d < 0] / sig_d)
            up += list(d[d > 0] / sig_b)
    n_del = P_DEL / 2**32 * total
    n_ben = P_BEN * 40 / 2**32 * total
    assert abs((total - same) - (n_del + n_ben)) < 5 * math.sqrt(n_del + n_ben)
    assert stats.kstest(dn, stats.halfnorm.cdf).pvalue > 1e-3
    assert len(up) > 20 and stats.kstest(up, stats.halfnorm.cdf).pvalue > 1e-3


def test_purifying_only_never_gains(orc):
    _, fit, ped = gens_with_pedigree(orc, 50, tournament=5, del_thr=P_DEL, ben_thr=0)
    for g in range(50):
        assert np.all(fit[g + 1] <= fit[g][ped[g]])
    assert fit[-1].max() <= 0.0 and fit[-1].min() < 0.0


def test_adaptive_rises_under_selection_not_neutral(orc):
    kw = dict(del_thr=P_DEL, ben_thr=P_BEN * 20, W=8, H=8, N=32, migrants=1)
    _, f5, _ = gens_with_pedigree(orc, 200, tournament=5, **kw)
    _, f0, _ = gens_with_pedigree(orc, 200, tournament=0, **kw)
    assert f5[-1].mean() > 0 > f0[-1].mean()


@pytest.mark.parametrize("bad", [dict(tournament=6), dict(del_thr=2**31, ben_thr=2**31 + 1),
                                 dict(del_sigma=-1.0), dict(ben_sigma=float("nan")),
                                 dict(del_sigma=1e7)])
def test_invalid_float_configs(orc, bad):
    kw = dict(tournament=5, del_thr=P_DEL, ben_thr=P_BEN, del_sigma=1.0, ben_sigma=1.0)
    kw.update(bad)
    with pytest.raises(ValueError):
        orc.Run(2, 2, 8, 32, 0, fitness_model=F, **kw)


def test_integer_model_rejects_other_tournaments(orc):
    with pytest.raises(ValueError):
        orc.Run(2, 2, 8, 32, 0, tournament=5)
