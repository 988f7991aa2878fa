"""Pins for the oracle's randomised single-term estimator (CPU only).

Sec. 7 cites Rhee and Glynn's extra randomisation that makes the multilevel
estimator unbiased.  Checked against:
  - the level draws recomputed in numpy from the oracle's (separately pinned)
    Philox words and the closed-form truncated geometric law, bit for bit,
    and a chi-square test of the counts against that law;
  - unbiasedness: with Milstein paths (beta = 2 > 1) the estimates over
    independent seeds average to the Black--Scholes price, with no finest
    level chosen, while a fixed coarse level shows its bias;
  - the reported per-sample variance against the spread over seeds.
"""
import numpy as np
import pytest
from scipy import stats

Q2 = 2.0 ** -1.5


def test_level_draws_bit_exact(orc):
    seed, N, Lc = 7, 4003, 12
    got = orc.rg_level_counts(seed, N, Q2, Lc)
    p = (1 - Q2) * Q2 ** np.arange(Lc + 1) / (1 - Q2 ** (Lc + 1))
    F = np.cumsum(p)
    F[-1] = 1.0
    counts = np.zeros(Lc + 1, np.uint64)
    for i in range(N):
        w = orc.path_words(seed, 0, i // 4, orc.STREAM_LEVEL_DRAW, 1)[i % 4]
        u = ((int(w) >> 8) + 0.5) * 2.0**-24
        counts[min(int(np.searchsorted(F, u, side="right")), Lc)] += 1
    assert np.array_equal(got, counts)
    pp, FF = orc.rg_probabilities(Q2, Lc)
    assert np.allclose(pp, p, rtol=1e-14) and abs(pp.sum() - 1) < 1e-14


def test_level_counts_follow_the_law(orc):
    N, Lc = 2_000_000, 10
    c = orc.rg_level_counts(3, N, 0.3, Lc).astype(float)
    p, _ = orc.rg_probabilities(0.3, Lc)
    keep = p * N > 20
    chi2 = (((c - N * p) ** 2) / (N * p))[keep].sum()
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-3, (c, N * p)


def test_unbiased_with_milstein(orc):
    m = orc.model(scheme=1)
    p = orc.payoff()
    bs = orc.bs_call()
    est, var = [], []
    for seed in range(1, 31):
        r = orc.rhee_glynn(m, p, 2, 15, Q2, 40000, seed, nthreads=8)
        est.append(r["estimate"])
        var.append(r["variance"])
    est = np.array(est)
    se = est.std(ddof=1) / np.sqrt(est.size)
    print("mean", est.mean(), "bs", bs, "se", se)
    assert abs(est.mean() - bs) < 4.5 * se
    # the reported per-sample variance matches the spread across seeds
    ratio = est.var(ddof=1) / (np.mean(var) / 40000)
    assert 0.5 < ratio < 2.0, ratio
    # a fixed two-level estimate has a visible bias at the same sample effort
    fixed = [orc.level(m, p, 0, 2, 40000, s, nthreads=8)["sum_y"] / 40000
             + orc.level(m, p, 1, 2, 40000, s, nthreads=8)["sum_y"] / 40000 for s in range(1, 31)]
    assert abs(np.mean(fixed) - bs) > 4.5 * np.std(fixed, ddof=1) / np.sqrt(30)


def test_bad_arguments(orc):
    with pytest.raises(ValueError):
        orc.rg_level_counts(1, 10, 1.5, 4)
    with pytest.raises(ValueError):
        orc.rg_level_counts(1, 10, 0.5, 16)
