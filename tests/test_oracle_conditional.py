"""Pins for the oracle's conditional digital (CPU only).

The payoff is the digital's expectation given every increment of a sample
but the last fine one (Sec. 7: conditional Monte Carlo inside the multilevel
estimator).  Checked against things other than its own formula:
  - Monte Carlo over the last increment: for a few samples, the plain
    digital of separately written fine and coarse paths, averaged over many
    redraws of the last fine increment, equals the conditional payoff;
  - the tower property on the same samples: plain minus conditional has
    mean zero at every level, for Euler and Milstein, GBM and Heston;
  - level 0 is deterministic: its value is the one-step digital, which the
    plain digital's level-0 mean over 10^6 samples reproduces;
  - what it buys: level variances far below the plain digital's, and with
    Milstein a decay rate well above the plain digital's one half.
"""
import numpy as np
import pytest

S0, K, R, SIG, T = 100.0, 100.0, 0.05, 0.2, 1.0
DISC = np.exp(-R * T)


def gbm_paths(dw, scheme):
    """Terminal values of GBM paths, one row of increments per path."""
    n = dw.shape[1]
    h = T / n
    S = np.full(dw.shape[0], S0)
    for i in range(n):
        f = 1.0 + R * h + SIG * dw[:, i]
        if scheme == 1:
            f = f + 0.5 * SIG * SIG * (dw[:, i] ** 2 - h)
        S = S * f
    return S


def digital(S):
    return DISC * np.where(S > K, 1.0, np.where(S == K, 0.5, 0.0))


@pytest.mark.parametrize("scheme", [0, 1])
def test_conditional_payoff_is_the_mean_over_the_last_increment(orc, scheme):
    m = orc.model(scheme=scheme)
    p = orc.payoff(kind=orc.DIGITAL_COND, K=K, payout=1.0)
    rng = np.random.default_rng(5)
    for M, l in ((2, 1), (2, 3), (4, 2)):
        nf = M**l
        h = T / nf
        pf, pc = orc.level_paths(m, p, l, M, 6, seed=3, offset=11)
        for i in range(6):
            dw = np.sqrt(h) * orc.path_normals(3, l, 11 + i, 0, 1, nf)
            n = 400000
            paths = np.tile(dw, (n, 1))
            paths[:, -1] = np.sqrt(h) * rng.standard_normal(n)   # redraw the last increment
            f = digital(gbm_paths(paths, scheme)).mean()
            c = digital(gbm_paths(paths.reshape(n, nf // M, M).sum(axis=2), scheme)).mean()
            tol = 4.5 * 0.5 / np.sqrt(n)
            assert abs(pf[i] - f) < tol, (M, l, i, pf[i], f)
            assert abs(pc[i] - c) < tol, (M, l, i, pc[i], c)


@pytest.mark.parametrize("kind,scheme", [(0, 0), (0, 1), (1, 0)])
def test_tower_property_on_the_same_samples(orc, kind, scheme):
    m = orc.model(kind=kind, scheme=scheme)
    plain = orc.payoff(kind=orc.DIGITAL, K=K, payout=1.0)
    cond = orc.payoff(kind=orc.DIGITAL_COND, K=K, payout=1.0)
    N = 100000
    for M, l in ((2, 0), (2, 2), (4, 1), (4, 3)):
        a = orc.level_paths(m, plain, l, M, N, seed=4, nthreads=8)
        b = orc.level_paths(m, cond, l, M, N, seed=4, nthreads=8)
        for x, y in zip(a, b):
            d = x - y
            assert abs(d.mean()) < 4.5 * d.std() / np.sqrt(N) + 1e-15, (M, l)


def test_level0_is_the_one_step_digital(orc):
    for scheme in (0, 1):
        m = orc.model(scheme=scheme)
        c = orc.level(m, orc.payoff(kind=orc.DIGITAL_COND), 0, 2, 1000, 1)
        assert abs(c["sum_y2"] / 1000 - (c["sum_y"] / 1000) ** 2) < 1e-12   # deterministic
        N = 1000000
        d = orc.level(m, orc.payoff(kind=orc.DIGITAL), 0, 2, N, 9, nthreads=8)
        mean = d["sum_y"] / N
        sd = np.sqrt(mean * (DISC - mean) / N)
        assert abs(mean - c["sum_y"] / 1000) < 4.5 * sd


def test_conditioning_reduces_level_variance(orc):
    N = 100000
    for scheme, gain in ((0, 10.0), (1, 100.0)):
        m = orc.model(scheme=scheme)
        vp, vc = [], []
        for l in range(3, 8):
            for kind, out in ((orc.DIGITAL, vp), (orc.DIGITAL_COND, vc)):
                r = orc.level(m, orc.payoff(kind=kind), l, 2, N, seed=6, nthreads=8)
                mu = r["sum_y"] / N
                out.append(r["sum_y2"] / N - mu * mu)
        vp, vc = np.array(vp), np.array(vc)
        print("scheme", scheme, "plain", vp, "conditional", vc)
        assert np.all(vp / vc > gain)
        if scheme == 1:
            beta = -np.polyfit(np.arange(3, 8), np.log2(vc), 1)[0]
            assert beta > 1.1, beta


def test_conditional_digital_arguments(orc):
    with pytest.raises(ValueError):
        orc.level(orc.model(), orc.payoff(kind=5), 1, 2, 10, 1)
